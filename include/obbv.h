/*
 * obbv.h -- C ABI of libobbv, the MI355X (gfx950) outer-volume engine for
 * variational hierarchical oriented bounding boxes (Wang, Hua, Xu, Huo, Bao,
 * "Variational Hierarchical Directed Bounding Box Construction for Solid Mesh
 * Models", arXiv 2203.10521).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Return value: OBBV_OK (0) or a negative OBBV_ERR_* code.  No C++ exception
 *   crosses this boundary.  obbv_last_error() returns a thread-local message for
 *   the last failing call of the calling thread.
 * - "device" pointers are HIP device allocations (for example torch tensors on
 *   cuda:0 under ROCm); "host" pointers are ordinary host memory.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Calls
 *   are stream ordered and asynchronous unless marked "synchronous".
 * - The caller owns every buffer it passes and the library never frees caller
 *   memory.  Scratch memory is a per-device library pool, grown on demand and
 *   returned to HIP by obbv_release().
 * - Calls that take scratch from the pool share it: on one device, issue them
 *   on one stream (or order them), from one host thread at a time.  Calls that
 *   overlap in time (several streams, several threads) race on the pool.  A
 *   planned launch (obbv_ov_plan_launch) uses only its plan's memory; the
 *   Lloyd driver splits its floods over streams of its own with a separate
 *   part of the pool for each.
 * - Meshes are closed, consistently oriented triangle meshes (Sec. 6 of the paper:
 *   the method handles solid models only): every directed edge (a, b) occurs
 *   once and its reverse (b, a) once; triangles are counter-clockwise seen from
 *   outside.  Vertices are float32 xyz triples, triangles int32 index triples.
 * - A box is (center, axes, half): row k of `axes` is the unit local axis k in
 *   world coordinates (right handed); local coordinates are x' = axes (x - center);
 *   the box is { |x'_k| <= half[k] }.  These are the 6 free parameters (centre
 *   and axes) plus the enclosure-determined extents of Sec. 4.2.1.
 */
#ifndef OBBV_H
#define OBBV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define OBBV_OK 0
#define OBBV_ERR_INVALID_ARG (-1)     /* bad pointer, size, count, NaN parameter */
#define OBBV_ERR_MESH_NOT_CLOSED (-2) /* a directed edge lacks its reverse       */
#define OBBV_ERR_MESH_NOT_ORIENTED (-3) /* a directed edge occurs twice, or the
                                           enclosed volume is not positive       */
#define OBBV_ERR_DEGENERATE (-4)      /* nothing to compute (e.g. empty cluster) */
#define OBBV_ERR_WORKSPACE (-5)       /* scratch limit exceeded                  */
#define OBBV_ERR_OOM (-6)             /* hipMalloc or a host allocation failed   */
#define OBBV_ERR_HIP (-7)             /* a HIP runtime call failed               */
#define OBBV_ERR_UNSUPPORTED (-8)     /* option not available on this device     */
#define OBBV_ERR_INTERNAL (-9)        /* unexpected host-side failure (a thread
                                         that could not start, ...)              */

/* ---- device status word bits (obbv_status) ---------------------------- */
#define OBBV_STATUS_NAN_BOX 0x1u      /* a box had a non-finite parameter        */
#define OBBV_STATUS_BAD_INDEX 0x2u    /* a triangle index was out of range       */
#define OBBV_STATUS_OVERFLOW 0x4u     /* a planned launch needed more scratch than
                                         it was sized for; its results are invalid */

/* ---- data types -------------------------------------------------------- */
typedef struct {
  const float* vertices;    /* device, [n_vertices][3] float32              */
  const int32_t* triangles; /* device, [n_triangles][3] int32, CCW outward  */
  int32_t n_vertices;
  int32_t n_triangles;
} obbv_mesh;

typedef struct {
  float center[3];
  float axes[9]; /* row major; row k = local axis k */
  float half[3];
} obbv_box;      /* 60 bytes, 4-byte aligned, no padding */

/* Options of the outer-volume estimator (Sec. 4.1; see obbv_outer_volume). */
typedef struct {
  int32_t R;          /* rays per face edge: R x R rays per cast axis, 1..32767 */
  uint32_t axis_mask; /* bit w set: cast along local axis w; 0 means 7 (all) */
  uint64_t seed;      /* SplitMix64 seed of the ray jitter                   */
  int32_t block_rays; /* rays of one LDS ray block (a power of two in [1024,
                         16384]); 0 = library choice                       */
  uint32_t flags;     /* reserved, must be 0                                 */
} obbv_ov_params;

/* ---- library ------------------------------------------------------------ */

/* Version string, static storage. */
const char* obbv_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* obbv_last_error(void);

/* Synchronous.  Waits for `stream`, reads and clears the device status word
 * (OBBV_STATUS_* bits) of the current device into *out_flags (host, nullable). */
int obbv_status(void* stream, uint32_t* out_flags);

/* Synchronous.  Frees the scratch pool of every device. */
int obbv_release(void);

/* ---- mesh staging ------------------------------------------------------ */

/* Synchronous.  Validates a mesh for the closed-solid requirement (Sec. 6):
 * indices in [0, n_vertices), every directed edge once with its reverse once,
 * enclosed volume sum(det[a, b, c]) / 6 > 0.  Runs on the device: the edges go
 * through a hash table of undirected edges counting both directions; the
 * volume terms are summed exactly in 64-bit fixed point (one power-of-two scale
 * per mesh, from its largest |coordinate|), so the result does not depend on
 * thread order.
 * out_report (host, nullable, 4 entries): [0] number of directed edges without
 * exactly one reverse (an edge (a, a) has none), [1] number of repeated
 * directed edges, [2] number of out-of-range indices, [3] unused (0).
 * *out_volume (host, nullable): the signed enclosed volume (float64; 0 when an
 * index is out of range).
 * Returns OBBV_OK, OBBV_ERR_MESH_NOT_CLOSED, OBBV_ERR_MESH_NOT_ORIENTED or
 * OBBV_ERR_INVALID_ARG. */
int obbv_validate_mesh(const obbv_mesh* mesh, int32_t* out_report, double* out_volume,
                       void* stream);

/* ---- outer volume (the hot path) ----------------------------------------- */

/* Outer volume OBV(X, O) of every box (Sec. 3, Eq. 4: the volume of the box
 * outside the solid), by the jittered parallel-ray estimator of Sec. 4.1:
 * for each cast axis w in axis_mask, an R x R grid of cells on the face
 * [-h_u, h_u] x [-h_v, h_v] ((u, v) = the other two local axes in cyclic
 * order), one ray per cell at (-h_u + (i + xi) du, -h_v + (j + eta) dv) parallel
 * to axis w, with (xi, eta) drawn by SplitMix64 from
 * (seed, box_key[b], w, i, j); the inside length of [-h_w, h_w] on each ray is
 * integrated from its signed crossings (Eq. 9 generalised to a line), and
 * OBV = V_box - mean_w sum_rays L du dv with V_box = 8 h0 h1 h2.
 * Ray-triangle tests are FP32 edge functions with a top-left ownership rule: a
 * ray that meets an edge shared by two triangles facing the same way exactly
 * (edge function 0 in FP32) crosses exactly one of them, so every ray counts
 * each sheet of the surface once (watertight).  Each crossing's inside length is
 * rounded to a multiple of 2^-22 of the slab and summed exactly in int64, so
 * the result does not depend on scheduling and is bitwise reproducible.
 *
 * meshes     host array of n_meshes mesh descriptors (device data), n_meshes >= 1
 * boxes      device, [n_boxes] obbv_box
 * box_mesh   device, [n_boxes] int32 mesh index per box; NULL = all mesh 0
 * box_key    device, [n_boxes] uint32 jitter key per box; NULL = box index
 * params     host; R in [1, 32767]
 * out_obv    device, [n_boxes] float64 outer volume per box
 * A box with a zero extent gets OBV 0; a box with a non-finite parameter gets
 * NaN and sets OBBV_STATUS_NAN_BOX (read it with obbv_status).  n_boxes = 0 is
 * a no-op.  The call never waits for the device (scratch is sized from the
 * arguments); an index out of range sets OBBV_STATUS_BAD_INDEX.
 */
int obbv_outer_volume(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                      const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                      const obbv_ov_params* params, double* out_obv, void* stream);

/* As obbv_outer_volume, with optional extra outputs (each nullable, device):
 * out_vin_axis  [n_boxes][3] float64 inside volume per cast axis (0 if not cast)
 * out_ray_q     [n_boxes][3][R][R] int32 per-ray inside fraction of the slab,
 *               in units of 2^-22 (L / (2 h_w) * 2^22, rounded per crossing)
 * out_ray_hits  [n_boxes][3][R][R] int32 crossing counts of each ray on the
 *               kept side: n_in + 65536 n_beyond, n_in = crossings inside the
 *               slab [-h_w, h_w], n_beyond = crossings past the slab face of the
 *               kept side (above +h_w, or below -h_w when the cast is mirrored)
 * out_side      [n_boxes][3] int32: 0 = crossings above the slab bottom were
 *               used, 1 = crossings below the slab top (mirrored cast); the
 *               kept side is the half prism with fewer triangles
 * The per-ray outputs are meant for tests and need n_boxes * 3 * R * R entries. */
int obbv_outer_volume_ex(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes,
                         const int32_t* box_mesh, const uint32_t* box_key, int32_t n_boxes,
                         const obbv_ov_params* params, double* out_obv, double* out_vin_axis,
                         int32_t* out_ray_q, int32_t* out_ray_hits, int32_t* out_side,
                         void* stream);

/* As obbv_outer_volume for one mesh, for boxes that come in groups sharing a
 * centre and axes -- the candidate moves of the Lloyd partition (Sec. 4.2.1,
 * Eq. 12) are such groups: every candidate is its box grown to enclose one more
 * triangle.  frames[f] is the union of group f (its centre, axes and the
 * largest half extents of its boxes); box_frame[b] names the group of box b.
 * The mesh is culled and transformed once per group, so each box only streams
 * the frame coordinates of the triangles that project into a face of its
 * group's frame.  The result is bitwise the one of
 * obbv_outer_volume with the same boxes and keys.  A box whose centre or axes
 * differ (bitwise) from its frame's, or that reaches outside it, or whose
 * box_frame is out of range, walks the whole mesh instead (same result).
 *
 * frames     device, [n_frames] obbv_box, 1 <= n_frames <= n_boxes
 * box_frame  device, [n_boxes] int32
 * other arguments as obbv_outer_volume (box_key nullable = box index).
 * The call waits for the device only when the frame lists could exceed
 * 2 GiB (48 bytes per frame and triangle), to size them. */
int obbv_outer_volume_grouped(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
                              int32_t n_boxes, const obbv_ov_params* params, const obbv_box* frames,
                              const int32_t* box_frame, int32_t n_frames, double* out_obv, void* stream);

/* Exact outer volume (Sec. 3, Eq. 4), the evaluator without quadrature or
 * jitter: for every box, V_box minus the volume of the solid inside it, found
 * by the divergence theorem along the box's local axis `axis` (0, 1 or 2) in
 * float64.  Each triangle's projection on the face perpendicular to `axis` is
 * clipped to the face rectangle, split by the two slab planes and its depth,
 * clamped to the slab, integrated over the pieces, with the sign of the
 * projected triangle's orientation.  Exact up to float64 rounding on closed,
 * consistently oriented meshes (the value is the same along every axis);
 * summed in a fixed order (bitwise deterministic).
 *
 * mesh     host struct, device arrays (as obbv_outer_volume)
 * boxes    device, [n_boxes] obbv_box, 0 <= n_boxes <= 65,535
 * out_obv  device, [n_boxes] float64
 * A box with a zero extent gets OBV 0; a box with a non-finite parameter or a
 * negative extent gets NaN and sets OBBV_STATUS_NAN_BOX; a triangle with an
 * out-of-range index sets OBBV_STATUS_BAD_INDEX and counts as absent.  Work is
 * O(n_boxes x n_triangles); scratch 8 bytes per box and 4,096 triangles.
 * Stream ordered. */
int obbv_outer_volume_exact(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t axis,
                            double* out_obv, void* stream);

/* The paper's central-projection estimator of the outer volume (Sec. 4.1,
 * Eq. 9-10): rays leave the box centre through the pixel centres of a
 * 6 x m x m cube map in the box frame; each pixel is a cone of directions of
 * its exact solid angle W.  A ray's crossings of the mesh (watertight test,
 * one owner for points on a shared edge) give the cone's outer volume
 * (r_e^3 - sum_k s_k min(r_k, r_e)^3) W / 3, r_e the distance at which the ray
 * leaves the box, r_k the crossing distances, s_k = +1 where the ray leaves the
 * solid and -1 where it enters (crossings beyond the box count as reaching
 * it); OBV is the sum over the cones.  A box inside the solid gives 0 exactly;
 * the estimate tends to the exact outer volume as m grows.  float64, fixed
 * summation order (bitwise deterministic).
 *
 * mesh     host struct, device arrays (as obbv_outer_volume)
 * boxes    device, [n_boxes] obbv_box, 0 <= n_boxes <= 65,535
 * m        pixels per cube-map face side, 1..256
 * out_obv  device, [n_boxes] float64
 * A box with a non-finite parameter or a negative extent gets NaN and sets
 * OBBV_STATUS_NAN_BOX; a triangle with an out-of-range index sets
 * OBBV_STATUS_BAD_INDEX and counts as absent.  Work is O(n_boxes x 6 m^2 x
 * n_triangles) (every triangle is tested against every ray); scratch 8 bytes
 * per box and 256 rays.  Stream ordered. */
int obbv_outer_volume_central(const obbv_mesh* mesh, const obbv_box* boxes, int32_t n_boxes, int32_t m,
                              double* out_obv, void* stream);

/* Synthetic collision queries, the stand-in for the paper's collision
 * experiment (Sec. 5: colliders against a model's hierarchy, counting
 * bounding-volume tests).  For every sphere the hierarchy is descended from
 * the root: a node is tested against the sphere (float64: the squared distance
 * from the centre to the box in its frame, sum_k max(|Q_k . (x - c)| - h_k,
 * 0)^2, against r^2); when the sphere overlaps it and it has children, they are
 * tested in order; an overlapped leaf is a hit.  Unused nodes are not tested.
 *
 * nodes      device, [n_nodes] obbv_box in level order: level l holds
 *            branching^l nodes, node j of level l has children branching*j ..
 *            branching*j + branching - 1 of level l + 1 (the layout of
 *            obbv_build_hierarchy and obbv_build_obb_tree)
 * node_used  device, [n_nodes] uint8, nullable (every node used)
 * levels     1..16; branching 1..64
 * spheres    device, [n_spheres][4] float32 (centre xyz, radius), 16-byte aligned
 * out_tests  device, [n_spheres] int32: sphere-box tests of each query
 * out_hits   device, [n_spheres] int32: overlapped leaves of each query
 * Stream ordered; no scratch. */
int obbv_collision_queries(const obbv_box* nodes, const uint8_t* node_used, int32_t levels, int32_t branching,
                           const float* spheres, int32_t n_spheres, int32_t* out_tests, int32_t* out_hits,
                           void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): obbv_outer_volume for one
 * mesh with every scratch byte in a fixed 32 MiB device array of the library
 * (one per device, held until the process ends); the call allocates nothing
 * and never waits for the device.  The caller passes inputs and outputs as for
 * obbv_outer_volume (box_key nullable = box index); results are bitwise those
 * of obbv_outer_volume.  out_status (device, nullable): the call ORs its
 * OBBV_STATUS_* bits there (else into a word of the fixed array, which
 * obbv_status does not read).  Returns OBBV_ERR_WORKSPACE when the boxes need
 * more scratch than the array holds (about 16 bytes per box, cast axis and
 * 4,608 triangles of the mesh, plus 128 bytes per box).  Calls on one device
 * share the array: calls that overlap in time on one device (different
 * streams) race and give wrong results; calls ordered on one stream are safe. */
int obbv_outer_volume_noalloc(const obbv_mesh* mesh, const obbv_box* boxes, const uint32_t* box_key,
                              int32_t n_boxes, const obbv_ov_params* params, double* out_obv,
                              uint32_t* out_status, void* stream);

/* ---- measurement ----------------------------------------------------------- */

/* Host.  enable != 0: every later obbv_outer_volume* call records a pair of HIP
 * events around its cast kernel (cull, LDS ray block, ray-triangle tests) on
 * the call's stream and adds to device counters the ray-triangle tests it
 * performs (a kept triangle against the rays of the cells its conservative cell
 * range covers in a ray block) and the bytes of its culling stream (48 bytes
 * per triangle-list entry per (axis, ray block) unit, and with a jitter table 8
 * bytes per ray of the block).  enable == 0 stops recording. */
int obbv_profile_enable(int enable);

/* Synchronous.  Sums the elapsed time of the recorded ray-test launches and
 * returns it with the launch count, the test count and the byte count, and the
 * time during which at least one recorded launch ran (out_busy_ms: the union of
 * the launches' intervals, which is less than the sum when launches on several
 * streams overlap), then clears the record.  Outputs are host pointers, each
 * nullable. */
int obbv_profile_read(double* out_test_ms, int64_t* out_launches, int64_t* out_tests, int64_t* out_bytes,
                      double* out_busy_ms);

/* ---- planned (graph-replayed) evaluations ------------------------------------ */

typedef struct obbv_ov_plan obbv_ov_plan; /* opaque */

/* Synchronous.  Plans repeated evaluations of the same argument pointers (the
 * contents of `boxes` may change between launches): with params->block_rays == 0
 * the LDS ray block is autotuned (2048, 4096 and 8192 rays timed; the choice is
 * cached per GPU architecture, R and size buckets); the scratch is sized from the
 * arguments (no device pass is needed: the pipeline keeps no per-triangle
 * records in device memory), and one evaluation is captured into a HIP graph.
 * `headroom` (>= 1) is accepted for compatibility and not needed.  The plan
 * owns its scratch; the caller's arrays must outlive it. */
int obbv_ov_plan_create(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes, const int32_t* box_mesh,
                        const uint32_t* box_key, int32_t n_boxes, const obbv_ov_params* params, double* out_obv,
                        double headroom, void* stream, obbv_ov_plan** out);

/* Asynchronous.  Replays the planned evaluation on `stream` (writes out_obv).  If
 * the boxes now need more scratch than planned, OBBV_STATUS_OVERFLOW is set
 * (read with obbv_status) and out_obv is not valid: plan again. */
int obbv_ov_plan_launch(obbv_ov_plan* plan, void* stream);

/* Host.  Chosen rays per ray block, sizes [cast items, cast units, scratch
 * bytes] and the autotuner's timings [2048, 4096, 8192 rays] in ms (0 when not
 * tuned; out_tuned_ms has 3 entries); each nullable. */
int obbv_ov_plan_info(obbv_ov_plan* plan, int32_t* out_block_rays, int64_t* out_sizes, float* out_tuned_ms);

int obbv_ov_plan_destroy(obbv_ov_plan* plan);

/* ---- covariance OBB fit -------------------------------------------------- */

/* Area-weighted covariance box of every triangle cluster: the box axes are the
 * principal directions of the cluster's surface (continuous-surface covariance,
 * the PCA split of top-down builders, Sec. 2), decreasing eigenvalue, e2 = e0 x e1,
 * largest-|component| of e0 and of e1 positive; the extents enclose the cluster's
 * vertices tightly (Sec. 4.2.1: the extents follow from the centre and axes).
 * The 3x3 eigenproblem is solved in float64 by cyclic Jacobi.
 *
 * mesh         host descriptor (device data)
 * tri_cluster  device, [n_triangles] int32 cluster id in [0, n_clusters) or -1 (ignored)
 * out_boxes    device, [n_clusters] obbv_box; an empty cluster gets center 0,
 *              identity axes, half 0
 * out_eigvals  device, [n_clusters][3] float64 (decreasing), nullable
 */
int obbv_fit(const obbv_mesh* mesh, const int32_t* tri_cluster, int32_t n_clusters,
             obbv_box* out_boxes, double* out_eigvals, void* stream);

/* ---- same-layer Lloyd clustering (Sec. 4.2.1) ----------------------------- */

typedef struct obbv_lloyd obbv_lloyd; /* opaque state, created and destroyed in pairs */

/* Learned ranking of flood candidates (all pointers device, owned by the caller). */
typedef struct {
  const float* mlp_params; /* [obbv_mlp_param_count()] trained ranker            */
  const float* volume;     /* [N][N][N] occupancy volume (obbv_occupancy_volume)  */
  const float* frame;      /* [10] frame of the volume                            */
  int32_t N;               /* volume edge (8 nb)                                  */
  int32_t verify_top;      /* in ordinary rounds, candidates per receiving box
                              evaluated exactly (smallest predicted change);
                              0 = decide on the predictions alone                 */
  float max_error;         /* rolling mean |predicted - exact| outer fraction of
                              the last 256 judged candidates above which the rest
                              of the Lloyd iteration evaluates every candidate
                              exactly                                             */
  int32_t judge_every;     /* every judge_every-th ranked flood round, a sample of
                              its candidates is evaluated exactly (on a stream
                              of the library's own, while the flood goes on) to
                              judge the ranker (>= 1)                             */
} obbv_surrogate;

typedef struct {
  int32_t R;              /* rays per face edge of every outer-volume evaluation */
  int32_t block_rays;     /* rays per LDS ray block (0 = library choice)          */
  uint64_t seed;          /* SplitMix64 seed of the ray jitter                    */
  int32_t pops_per_round; /* K: frontier triangles taken per group per round; 1 = the
                             serial flood of the paper                            */
  int32_t reserved;       /* must be 0                                            */
  double delta;           /* rotation step (radians) of the parameter update      */
} obbv_lloyd_params;

/* Synchronous.  Copies the mesh to the host (the flood's queue and adjacency
 * live there; every outer volume is evaluated on the device) and creates a state.
 * The mesh's device arrays must stay valid while the state exists. */
int obbv_lloyd_create(const obbv_mesh* mesh, const obbv_lloyd_params* params, obbv_lloyd** out);

/* Host.  Defines the groups of one layer: tri_group[t] (host, [n_triangles]) is
 * the group of triangle t or -1; box b belongs to group box_group[b] (host,
 * [n_boxes]) and starts with centre and axes from boxes[b] (host, [n_boxes][15],
 * obbv_box layout; the half extents are ignored); box_slot[b] (host, nullable)
 * is its ray-jitter key (default b).  The boxes of a group partition its
 * triangles (Eq. 11). */
int obbv_lloyd_set_groups(obbv_lloyd* st, int32_t n_boxes, const int32_t* tri_group, const int32_t* box_group,
                          const float* boxes, const uint32_t* box_slot);

/* Synchronous.  One Lloyd iteration of every group: the flooding partition
 * (Sec. 4.2.1 step 1, Eq. 12-13) with the current centres and axes fixed, then
 * the parameter update of every box (step 2: tight box, finite-difference
 * rotation gradient, line search, kept if OBV drops). */
int obbv_lloyd_step(obbv_lloyd* st, void* stream);

/* Synchronous, like obbv_lloyd_step.  The adjustment of Sec. 4.2.1 (third step:
 * when the iteration stalls in a local minimum, the least important box is
 * adjusted and the result kept only if the error drops), for every group with
 * two boxes or more.  Reading of importance: the number of triangles a box
 * holds; ties go to the box with the larger outer volume, then the higher box
 * index.  The least important box moves to the centroid of the triangle
 * farthest from the centre of the group's box with the largest outer volume
 * (ties: lower box index, lower triangle index) and takes that box's axes; one
 * Lloyd iteration of the adjusted groups follows (as obbv_lloyd_step), and a
 * group keeps it only if the sum of its boxes' outer volumes is lower than
 * before, else its boxes, outer volumes and assignments are restored.  Groups
 * that were not adjusted are left unchanged.  Call after obbv_lloyd_step; the
 * caller decides when the iteration has stalled.
 * out_accepted (host, nullable, [number of groups]): 1 kept, 0 undone, -1 not
 * adjusted (fewer than two boxes, or the worst box holds no triangle). */
int obbv_lloyd_adjust(obbv_lloyd* st, int32_t* out_accepted, void* stream);

/* Host.  With a non-NULL surrogate, later flood rounds predict the outer
 * fraction f of every candidate box (a box grown by a popped triangle that no box
 * of its group contains) and of the current boxes, with the predicted change
 * dOBV = max(0, f(grown) V(grown) - f(current) V(current)) (Eq. 12).  In an
 * ranked round, of the candidates a box receives only the verify_top with the
 * smallest predicted change are evaluated exactly, and every triangle goes to
 * the box with the smallest change (exact where evaluated, predicted elsewhere);
 * a round with nothing to verify makes no outer-volume call on the caller's
 * stream.  Every judge_every-th ranked round also sends up to 256 of its
 * candidates (evenly strided) to an exact evaluation on a second stream, which
 * runs while the flood goes on; at the next such round (or the end of the flood)
 * its errors |predicted - exact| outer fraction enter a rolling mean over the
 * last 256: above max_error the rest of that iteration is exact (counted as a
 * fallback).  The judged rounds and the rounds at which their errors count do
 * not depend on timing, so a build is reproducible.  The outer volumes of grown boxes, the final boxes of the flood
 * and the parameter update stay exact.  NULL returns to exact evaluation of
 * every candidate.  The structure is copied; its device arrays must stay valid. */
int obbv_lloyd_set_surrogate(obbv_lloyd* st, const obbv_surrogate* surrogate);

/* Host.  Results of the last step (each output nullable, host):
 * tri_box [n_triangles] box of each triangle (-1 = none), boxes [n_boxes][15],
 * obv [n_boxes], *layer_error = sum of OBV (Eq. 6), counters [4] = outer-volume
 * evaluations, flood rounds, candidates that needed no evaluation, moves,
 * ranker predictions, ranker fallbacks to exact evaluation (counters has 6
 * entries, cumulative over the state's steps). */
int obbv_lloyd_get(obbv_lloyd* st, int32_t* tri_box, float* boxes, double* obv, double* layer_error,
                   int64_t* counters);

/* Host.  cap > 0: from now on the state keeps a uniform sample (reservoir of
 * size cap, drawn with SplitMix64) of the (box, exact outer volume) pairs it
 * evaluates -- flood candidates, grown boxes and parameter-update trials --
 * the training pairs of the learned ranker.  cap = 0 stops recording.  Either
 * call clears the sample. */
int obbv_lloyd_record(obbv_lloyd* st, int64_t cap);

/* Host.  Copies up to max_n recorded pairs (boxes [n][15] in obbv_box layout,
 * obv [n] float64; host arrays) and the count to *n_out, then clears the sample. */
int obbv_lloyd_take_records(obbv_lloyd* st, int64_t max_n, float* boxes, double* obv, int64_t* n_out);

int obbv_lloyd_destroy(obbv_lloyd* st);

/* ---- hierarchy (Sec. 4.2.2) ---------------------------------------------- */

typedef struct {
  int32_t levels;         /* layers including the root, 1..12                    */
  int32_t branching;      /* children per node, fixed in advance                  */
  int32_t iters;          /* Lloyd iterations per layer and pass                  */
  int32_t sweeps;         /* bottom-up / top-down sweeps after the first top-down */
  int32_t R;
  int32_t block_rays;
  int32_t pops_per_round;
  int32_t reserved;       /* must be 0 */
  uint64_t seed;          /* ray jitter and seed-triangle draws                   */
  double delta;
  const obbv_surrogate* surrogate; /* host pointer, NULL = exact evaluation only   */
} obbv_hier_params;

/* Synchronous.  Builds the hierarchy: the root is the covariance box of the mesh
 * refined by parameter updates; each lower layer splits every node's triangles
 * among `branching` children by same-layer Lloyd (top-down decomposition); each
 * sweep then merges layers bottom-up with the child boxes as units and keeps a
 * merge only if the hierarchy error e (Eq. 7, layer weight = number of layers to
 * the leaves, leaf = 1, Sec. 5) drops, and re-solves the layers below top-down,
 * again keeping only improvements.  Node numbering is level-major:
 * n_nodes = sum_l branching^l.  Outputs (host, each nullable):
 * out_boxes [n_nodes][15]; out_obv [n_nodes]; out_parent [n_nodes] (-1 root);
 * out_tri_node [levels][n_triangles] node of every triangle per layer;
 * out_e [1 + sweeps] e after the top-down pass and after every sweep;
 * out_counters [6] as obbv_lloyd_get. */
int obbv_build_hierarchy(const obbv_mesh* mesh, const obbv_hier_params* params, float* out_boxes, double* out_obv,
                         int32_t* out_parent, int32_t* out_tri_node, double* out_e, int64_t* out_counters,
                         void* stream);

/* ---- top-down OBB tree (comparison baseline) ------------------------------ */

/* Synchronous.  The top-down covariance-box tree the paper compares its
 * hierarchy with (Sec. 5, Fig. 6: OBB-tree style builders): the root box is the
 * covariance box of all triangles (obbv_fit); every node's triangles are ordered
 * by the projection of their centroids (float64) on the longest axis of the
 * node's box (ties by triangle index) and cut into `branching` parts of equal
 * count (part = rank * branching / count), each again fitted, down to `levels`
 * layers (root included, 1..12; branching 2..64).  Node numbering, outputs and
 * layouts as obbv_build_hierarchy: out_boxes [n_nodes][15], out_parent
 * [n_nodes], out_tri_node [levels][n_triangles] (host, each nullable). */
int obbv_build_obb_tree(const obbv_mesh* mesh, int32_t levels, int32_t branching, float* out_boxes,
                        int32_t* out_parent, int32_t* out_tri_node, void* stream);

/* ---- learned ranker of candidate boxes -------------------------------------- */

/* Occupancy features of boxes: for every box, 8 x 8 rays along local axis 2
 * (one jittered ray per cell, SplitMix64 seed `seed`, jitter key = box index),
 * and on each ray the inside length within each of the 8 equal sub-slabs of
 * [-h2, h2] divided by the sub-slab length (Sec. 4.1 integration on a coarse
 * grid).  Output row b of out_X (device, [n_boxes][544] float32):
 * [0..2] (centre - frame centre) / frame diagonal, [3..11] axes,
 * [12..14] log(half / frame diagonal), [15..526] occupancy (x-major, then y,
 * then z), [527..543] 0.  mesh_frame (device, [n_meshes][4]) = bounding-box
 * centre xyz and diagonal of each mesh. */
int obbv_box_features(const obbv_mesh* meshes, int32_t n_meshes, const obbv_box* boxes, const int32_t* box_mesh,
                      int32_t n_boxes, const float* mesh_frame, uint64_t seed, float* out_X, void* stream);

/* Occupancy volume of a mesh: an (8 nb)^3 grid of voxels over the box
 * frame[0..2] + [0, 8 nb) * frame[3..5] (origin, voxel size; device frame [10]),
 * filled with the sub-slab inside fractions of nb^3 axis-aligned tiling boxes
 * (obbv_box_features occupancy, jitter key = tiling box index).  out_volume:
 * device [8 nb][8 nb][8 nb] float32, index [z][y][x].  frame[6..9] (bounding-box
 * centre xyz and diagonal) is used by obbv_sample_features. */
int obbv_occupancy_volume(const obbv_mesh* mesh, int32_t nb, const float* frame, uint64_t seed, float* out_volume,
                          void* stream);

/* Ranker input rows sampled from an occupancy volume (the fast path used inside
 * the Lloyd flood): [0..14] as obbv_box_features (normalised by frame[6..9]);
 * [15..526] the volume at the 8 x 8 x 8 sub-cell centres of the box (trilinear,
 * voxel centres at origin + (i + 1/2) voxel, 0 outside), x-major then y then z. */
int obbv_sample_features(const float* volume, int32_t N, const float* frame, const obbv_box* boxes, int32_t n_boxes,
                         float* out_X, void* stream);

/* Number of float32 parameters of the ranker MLP (544 -> 256 -> 256 -> 1):
 * W1 [544][256], b1 [256], W2 [256][256], b2 [256], w3 [256], b3 [1], in this
 * order; W[i][o] multiplies input i into output o. */
int64_t obbv_mlp_param_count(void);

/* Predicted outer fraction OBV / V_box of n rows (device X [n][544], out_f [n]);
 * n a multiple of 32.  The network corrects the occupancy estimate:
 * f = (1 - mean of X[15..526]) + sigmoid(z) - 1/2, z the MLP output.  Products
 * on bfloat16 MFMA with float32 accumulation. */
int obbv_mlp_forward(const float* params, const float* X, int32_t n, float* out_f, void* stream);

/* Predicted outer fraction of n_boxes boxes in one launch: the input rows of
 * obbv_sample_features are built on chip and fed to the network of
 * obbv_mlp_forward; out_f (device or mapped host [n_boxes], any n_boxes >= 0)
 * receives the same bits as obbv_sample_features followed by obbv_mlp_forward.
 * `boxes` may be device memory or mapped pinned host memory (each box is read
 * once).  Used by the Lloyd flood's ranked rounds. */
int obbv_mlp_rank_boxes(const float* params, const float* volume, int32_t N, const float* frame,
                        const obbv_box* boxes, int32_t n_boxes, float* out_f, void* stream);

/* One training step on n rows (multiple of 32): forward, mean squared error
 * against target (device [n]), backward, Adam update (lr > 0; step counts from
 * 1; adam_m / adam_v device [param_count], zero before the first step).
 * out_loss (device [1], nullable) receives the loss before the update;
 * out_grad (device [param_count], nullable) the gradient.  lr = 0 computes the
 * gradient without updating. */
int obbv_mlp_train_step(float* params, float* adam_m, float* adam_v, int32_t step, const float* X, const float* target,
                        int32_t n, float lr, float* out_loss, float* out_grad, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OBBV_H */
