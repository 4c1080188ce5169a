/*
 * rgg.h -- C ABI of librgg: Red-Green-Gray classification of roadmap edges
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method (Arad et al., "Serialized Red-Green-Gray: Quicker Heuristic
 * Validation of Edges in Dynamic Roadmap Graphs"):
 *   Sec. 4.1   an edge whose inner approximation meets an obstacle is RED,
 *              one whose outer approximation misses every obstacle is GREEN,
 *              any other edge is GRAY (unknown, left for a full check);
 *   Sec. 3.2   cfg(e) = |e|/eps configurations along the edge; an outer
 *              (inner) approximation is a superset (subset) of the swept
 *              volume;
 *   Alg. 1     when an obstacle moves, only the components it touched before
 *              and touches now are revisited;
 *   Sec. 4.3   the approximations are stored once, resident on the GPU, and
 *              only the new obstacle poses go up per update; a uniform grid
 *              restricts the tests to edges near the moved obstacles.
 *
 * Primitives of this library:
 *   robot       a union of spheres on a planar rigid body (SE2: x, y, theta),
 *               a spatial rigid body (SE3: x, y, z, qw, qx, qy, qz) or a planar
 *               serial arm (joint angles q0..q_{L-1});
 *   inner       the robot's spheres at every configuration of cfg(e), or
 *               (rgg_build_opts.inner_splines, Sec. 4.2) each sphere's
 *               shortcut spline through its centres, thickened to stay in
 *               the swept volume;
 *   outer       per sphere, a capsule around the chord of its centre path,
 *               radius r_i + delta_i with delta_i = max|p''| / 8 (the
 *               linear-interpolation error bound of the centre path), and
 *               optionally (rgg_build_opts.outer_obb, Sec. 4.2) intersected
 *               with an oriented box around its body's sweep;
 *   obstacles   closed axis-aligned boxes.
 *
 * Conventions for every entry point:
 *   - Every call returns an rgg_status: RGG_OK (0) or a negative error code.
 *     After an error, rgg_last_error() gives a message for the calling thread.
 *   - The caller owns every pointer it passes.  The library copies what it
 *     keeps (robot, approximations, resident obstacle slots); no host array
 *     is retained after a call returns.
 *   - Host pointers are plain CPU memory; "device" pointers are GPU memory of
 *     the context's device (e.g. torch tensors' data_ptr()).
 *   - A roadmap is not thread-safe: calls on one roadmap must not overlap.
 *     Different roadmaps may be used from different threads.
 */
#ifndef RGG_H
#define RGG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rgg_status;
#define RGG_OK 0
#define RGG_E_INVALID_ARG (-1)     /* bad argument; nothing changed          */
#define RGG_E_OUT_OF_MEMORY (-2)   /* host or device allocation failed       */
#define RGG_E_STATE_MISMATCH (-3)  /* `old` differs from the resident slots  */
#define RGG_E_CAPACITY (-4)        /* gray list longer than the caller's cap */
#define RGG_E_DEVICE (-5)          /* HIP runtime error                      */
#define RGG_E_UNSUPPORTED (-6)     /* valid request the library cannot serve */
#define RGG_E_BUSY (-7)            /* server queue full; submit again later  */

/* robot kinds */
#define RGG_SE2 0
#define RGG_SE3 1
#define RGG_PLANAR_ARM 2

/* labels, one uint8_t per edge */
#define RGG_GREEN 0
#define RGG_GRAY 1
#define RGG_RED 2

/* verdicts of the full validation (rgg_validate) */
#define RGG_VERDICT_FREE 0        /* no configuration of the motion collides     */
#define RGG_VERDICT_COLLIDES 2    /* a witness configuration collides           */
#define RGG_VERDICT_UNRESOLVED 3  /* undecided within the refinement limits     */
#define RGG_VERDICT_BAD_ID 255    /* the listed id is not an edge of the roadmap */

/* precision of the distance tests */
#define RGG_PREC_FP64 0           /* every test in binary64                   */
#define RGG_PREC_FP32_RECHECK 1   /* binary32 tests; any pair with a margin in
                                     the rounding band is re-tested in
                                     binary64, so labels equal the FP64 ones */

/* rgg_build_opts.inline_rounds: how the FP32 mode splits the pair tests
 * between the blocks that list an item's pairs and the balanced pair testing */
#define RGG_INLINE_ALL 0          /* every round (one fused kernel; default)   */
#define RGG_INLINE_NONE (-1)      /* no round (every pair listed)              */

/* A closed axis-aligned box.  Planar roadmaps use indices 0 and 1; indices 2
 * must still be finite.  A box with lo[k] > hi[k] on any used axis is ABSENT:
 * it meets nothing.  The canonical ABSENT box, held by every slot after
 * rgg_build, is lo = {1,1,1}, hi = {-1,-1,-1}. */
typedef struct {
    double lo[3];
    double hi[3];
} rgg_box;

typedef struct {
    int32_t kind;                 /* RGG_SE2 / RGG_SE3 / RGG_PLANAR_ARM        */
    int32_t n_spheres;            /* B, 1..64                                   */
    int32_t n_links;              /* arm only, 1..32                            */
    int32_t reserved;
    const double *sphere_pos;     /* SE2 [B][2], SE3 [B][3] body-frame offsets;
                                     arm [B] distance along the sphere's link   */
    const int32_t *sphere_link;   /* arm only: [B] link index of each sphere    */
    const double *sphere_radius;  /* [B], > 0                                   */
    const double *link_length;    /* arm only: [n_links]                        */
    double base[2];               /* arm only: base position                    */
} rgg_robot;

typedef struct {
    int64_t n_nodes;
    const double *q;              /* [n_nodes][dof] host, dof = 3 / 7 / n_links;
                                     SE3 quaternions (qw,qx,qy,qz) unit length   */
    int64_t n_edges;
    const int64_t *edge_uv;       /* [n_edges][2] host node ids; the caller's
                                     edge order is the order of every output.
                                     An edge (v, v) is node v (Sec. 3.1: a node
                                     is a degenerate edge): its one configuration
                                     gives node v's label, RED or GREEN, never
                                     GRAY                                       */
} rgg_roadmap_desc;

typedef struct {
    double resolution;            /* eps, C-space step between configurations */
    int32_t samples_per_edge;     /* > 1 fixes |cfg(e)|, overriding resolution  */
    int32_t precision;            /* RGG_PREC_*                                 */
    double band_rel;              /* FP32 band factor tau: a test whose FP32
                                     margin m (squared distance minus squared
                                     radius) has |m| <= tau (s + R)(R + L)
                                     + tau^2 s^2 is decided in FP64, where s is
                                     the largest |coordinate| of the pair, R
                                     the radius tested and L the L1 length of
                                     the capsule axis (0 for a sphere copy).
                                     <= 0 selects 1e-5; +inf re-tests every
                                     pair.  The FP32 rounding error is below
                                     28 u s (R + L) + 7 u R^2 (u = 2^-24), so
                                     labels do not depend on it for any value
                                     >= 2^-18.                                  */
    int64_t n_obstacle_slots;     /* M, 0..4096                                 */
    double cell_size;             /* grid cell edge; 0 = heuristic; < 0 = one
                                     cell covering everything                   */
    int32_t host_threads;         /* threads for the host build; 0 = automatic  */
    int32_t retest_capacity;      /* FP32 mode: undecided pairs each item block
                                     (at most 2048 of them) may queue for the
                                     binary64 re-test, over all the items it
                                     takes of this roadmap in one update,
                                     before it leaves a whole work item to the
                                     binary64 pass instead; 0 = 1024, at most
                                     2^20.  Any value gives the same labels.   */
    int32_t item_edges;           /* edges per work item of the classify
                                     kernels (one block of 256 threads each,
                                     up to two edges per thread), 1..512;
                                     0 = 256.
                                     rgg_tune may change it.  Any value gives
                                     the same labels.                           */
    int32_t outer_obb;            /* 1: the second outer form of Sec. 4.2 as
                                     well: an oriented box per robot body (the
                                     whole robot for SE2/SE3, a link for the
                                     arm) on the principal axes of the body's
                                     sphere centres along the edge, widened to
                                     hold the continuous sweep; a sphere's
                                     outer part is its capsule intersected with
                                     its body's box, tested by the separating-
                                     axis theorem in binary64.  0: capsules
                                     only.                                      */
    int32_t inner_splines;        /* 1: the second inner form of Sec. 4.2: each
                                     sphere's spline through its centres,
                                     simplified by Agarwal et al.'s greedy
                                     shortcuts (error err <= spline_tol * r_i),
                                     each kept segment a capsule of radius
                                     r_i - err - delta_i / n^2, which stays in
                                     the swept volume, replaces the sphere's
                                     copies.  0: copies                         */
    double spline_tol;            /* shortcut tolerance, a fraction of the
                                     sphere's radius in (0, 1); 0 selects 0.05 */
    int32_t pair_list_capacity;   /* FP32 mode with pair listing (see
                                     inline_rounds): pairs each of the 2048
                                     listing blocks may hand to the balanced
                                     pair testing (rounds that do not fit it
                                     tests itself); 0 = 512, at most 2^20.  Any
                                     value gives the same labels                */
    int32_t inline_rounds;        /* FP32 mode: pair rounds (of up to 256 pairs)
                                     of each work item that its listing block
                                     tests itself before it lists the rest for
                                     the balanced pair testing.  RGG_INLINE_ALL
                                     (0, the default) = every round: one fused
                                     kernel, no pair lists allocated, the pair
                                     testing not launched; n > 0 = the first n
                                     rounds (at most 2^20); RGG_INLINE_NONE =
                                     none, every round listed.  Any value gives
                                     the same labels                            */
    int64_t mem_budget;           /* device bytes the roadmap may hold; 0 = the
                                     free device memory.  A roadmap whose arrays
                                     would need more (rgg_roadmap_info's
                                     device_bytes) is refused with
                                     RGG_E_OUT_OF_MEMORY before anything is
                                     allocated; a budget above the free memory
                                     admits up to the free memory               */
} rgg_build_opts;

/* Written by the device at the end of every update (rgg_update_async) and
 * returned by rgg_update. */
typedef struct {
    int32_t status;               /* RGG_OK, RGG_E_INVALID_ARG (non-finite box)
                                     or RGG_E_STATE_MISMATCH; on error nothing
                                     changed and no output was written          */
    int32_t n_changed;            /* changed (box, sign) entries this update    */
    int64_t n_gray;               /* number of GRAY edges (may exceed gray_cap) */
    int64_t n_candidate_edges;    /* edges passing the grid + box pretest       */
    int64_t n_pairs;              /* (edge, changed box) pairs tested           */
    int64_t n_outer_hits;         /* pairs whose outer approximation met        */
    int64_t n_rechecked;          /* pairs re-decided in binary64               */
    int64_t n_cells_visited;      /* (cell, edge) entries scanned by the grid   */
    int64_t test_bytes;           /* bytes the classify kernels read and wrote:
                                     the item kernel, the balanced pair testing
                                     and the binary64 pass together             */
    int64_t item_bytes;           /* the FP32 item kernel's part of test_bytes
                                     (its pair listing and inline pair tests)   */
    int64_t fp64_bytes;           /* the binary64 pass's part of test_bytes     */
} rgg_update_result;

typedef struct {
    int64_t n_edges;
    int64_t n_slots;
    int32_t dim;                  /* workspace dimension D (2 or 3)             */
    int32_t n_spheres;
    int64_t n_sphere_samples;     /* sum over edges of |cfg(e)| * B             */
    int64_t grid_cells[3];
    double cell_size;
    int64_t grid_entries;         /* (cell, edge) registrations                 */
    int64_t device_bytes;         /* device memory held by the roadmap          */
    double build_seconds;
    int32_t item_edges;           /* edges per work item                         */
} rgg_roadmap_info;

typedef struct rgg_context rgg_context;
typedef struct rgg_roadmap rgg_roadmap;
typedef struct rgg_graph rgg_graph;
typedef struct rgg_batch rgg_batch;

/* Opens `device` (HIP ordinal) for later builds.  *out receives the context. */
rgg_status rgg_context_create(int device, rgg_context **out);
void rgg_context_destroy(rgg_context *ctx);

/* Builds the approximations of every edge (Sec. 4.3 offline storage: built
 * once, resident on the GPU): FP64 forward kinematics at every configuration
 * of cfg(e) (Sec. 3.2), per-sphere capsules, edge bounding boxes and the
 * uniform grid (Sec. 4.3 spatial filtering).  Every obstacle slot starts
 * ABSENT, so every label starts GREEN (Sec. 5: roadmaps are built without
 * obstacles).  Errors: RGG_E_INVALID_ARG (null pointer, node id out of
 * range, non-finite or non-unit input, bad option), RGG_E_OUT_OF_MEMORY,
 * RGG_E_DEVICE.  *out receives the roadmap. */
rgg_status rgg_build(rgg_context *ctx, const rgg_roadmap_desc *roadmap, const rgg_robot *robot,
                     const rgg_build_opts *opts, rgg_roadmap **out);
rgg_status rgg_destroy(rgg_roadmap *rm);
rgg_status rgg_roadmap_info_get(rgg_roadmap *rm, rgg_roadmap_info *out);

/* One update (Alg. 1 for every slot whose box changed, Sec. 4.1 labels),
 * host buffers.  `obstacles_old` and `obstacles_new` are [m] host boxes;
 * m must equal n_obstacle_slots and `obstacles_old` must equal the resident
 * slots bit for bit (else RGG_E_STATE_MISMATCH, nothing changes).  Slots
 * whose old and new boxes differ are the moved obstacles; adding and removing
 * go through ABSENT.  After the call the labels of all edges equal the rule
 * applied to `obstacles_new`.  Outputs (each may be NULL): labels [E] host,
 * gray [gray_cap] host (ascending GRAY edge ids), *n_gray, *result.  If
 * n_gray > gray_cap the update is still committed, gray[0..gray_cap) is
 * written and RGG_E_CAPACITY is returned.  Blocks until done. */
rgg_status rgg_update(rgg_roadmap *rm, int64_t m, const rgg_box *obstacles_old,
                      const rgg_box *obstacles_new, uint8_t *labels, int64_t *gray,
                      int64_t gray_cap, int64_t *n_gray, rgg_update_result *result);

/* The same update with every buffer in device memory, queued on `stream`
 * (a hipStream_t; NULL = the null stream) and returning at once.
 * d_old/d_new [m] boxes, d_labels [E] (or NULL), d_gray [gray_cap] (or NULL),
 * d_result (required) receive the outputs in stream order.  Validation of the
 * boxes happens on the device: on a bad box or a state mismatch
 * d_result->status is set, nothing changes and no label or gray id is
 * written.  Host-side errors (bad pointers, m != slots) return at once. */
rgg_status rgg_update_async(rgg_roadmap *rm, void *stream, int64_t m, const rgg_box *d_old,
                            const rgg_box *d_new, uint8_t *d_labels, int64_t *d_gray,
                            int64_t gray_cap, rgg_update_result *d_result);

/* A request for rgg_graph_create: the arguments of one rgg_update_async. */
typedef struct {
    rgg_roadmap *rm;
    int64_t m;
    const rgg_box *d_old, *d_new;
    uint8_t *d_labels;
    int64_t *d_gray;
    int64_t gray_cap;
    rgg_update_result *d_result;
} rgg_update_req;

/* Captures n updates into one HIP graph: requests naming the same roadmap run
 * in the order given, requests on different roadmaps run as independent
 * branches.  Every launch of the graph performs all n updates; the device
 * pointers are fixed at creation.  *out receives the graph. */
rgg_status rgg_graph_create(rgg_context *ctx, int32_t n, const rgg_update_req *reqs,
                            rgg_graph **out);
rgg_status rgg_graph_launch(rgg_graph *g, void *stream);
rgg_status rgg_graph_destroy(rgg_graph *g);

/* Batched updates of many roadmaps (at most 256, distinct, one device): one
 * update of each roadmap per launch, all of them in a single captured graph
 * whose kernels each process every roadmap of the batch (one launch per
 * stage, not per roadmap; roadmaps of the same robot dimension and precision
 * share one item kernel over the union of their work items).  Each update
 * computes exactly what rgg_update_async computes for its roadmap.
 *
 * rgg_batch_create fixes the roadmaps (rms[n]).  rgg_batch_launch queues one
 * batched update on `stream` (the stage kernels launched in stream order;
 * rgg_batch_launch_graph launches them as the captured graph instead):
 * reqs[n] gives, in the same order, each
 * roadmap's update arguments (reqs[k].rm must equal rms[k]); their device
 * pointers may differ from launch to launch, since the request table is
 * read from pinned host memory by the launch's first kernel, in stream
 * order.
 * Errors: RGG_E_INVALID_ARG (null pointer, n out of range, a repeated
 * roadmap, another device, a request that does not match its roadmap),
 * RGG_E_DEVICE.  Device-side errors (bad box, state mismatch) are reported
 * per request in its d_result, as for rgg_update_async.  A batch must be
 * destroyed before any of its roadmaps; rgg_batch_destroy waits for its
 * launches to finish. */
rgg_status rgg_batch_create(rgg_context *ctx, int32_t n, rgg_roadmap *const *rms, rgg_batch **out);
rgg_status rgg_batch_launch(rgg_batch *b, const rgg_update_req *reqs, void *stream);
/* The same batched update as one launch of the batch's captured graph. */
rgg_status rgg_batch_launch_graph(rgg_batch *b, const rgg_update_req *reqs, void *stream);
rgg_status rgg_batch_destroy(rgg_batch *b);
/* Stage timing of rgg_batch_launch (not of the graph form), with HIP events
 * on the launch's stream: rgg_batch_timing_read returns the summed
 * milliseconds of each stage over the launches since the last read and
 * resets them: ms[0] diff, ms[1] grid cells, ms[2] 0, ms[3] the item kernels,
 * ms[4] the binary64 pass, ms[5] labels and gray lists.  It waits for the
 * timed launches. */
rgg_status rgg_batch_timing_enable(rgg_batch *b, int32_t on);
rgg_status rgg_batch_timing_read(rgg_batch *b, double ms[6], int64_t *n_launches);

/* One batched update of n distinct roadmaps (create, launch, wait, destroy):
 * the convenience form of the three calls above.  Blocks until done. */
rgg_status rgg_update_batch(rgg_context *ctx, int32_t n, const rgg_update_req *reqs, void *stream);

/* For callers that cannot allocate memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it): the
 * batched update of rgg_update_batch, computing the same results, with the
 * request table in a fixed device array that the library holds (one per
 * device, up to 256 requests, 121 KiB, kept until the process ends)
 * instead of a batch created per call.  Calls no allocator: no hipMalloc,
 * hipFree, pinned or pageable host allocation, graph or event creation.
 * Arguments as rgg_update_batch (device pointers in reqs, queued on
 * `stream`); blocks until the update is done.  Errors: RGG_E_INVALID_ARG
 * for n outside 1..256 (the table's capacity), a null pointer, a repeated
 * roadmap, another device or a request that does not match its roadmap,
 * with nothing queued; RGG_E_DEVICE.  Every context of a device shares that
 * device's table, which keeps the last call's rows; calls from one process
 * are serialised by the library (each waits for the previous to finish),
 * and nothing in the table needs to start at zero. */
rgg_status rgg_update_batch_noalloc(rgg_context *ctx, int32_t n, const rgg_update_req *reqs, void *stream);

/* Autotuner of the work decomposition (Sec. 4.3 sizes grid cells by what
 * one kernel can process; here the choice is made by measurement).  The
 * candidates are the roadmap's current configuration, every combination
 * of work-item size (512, 256, 128 or 64 edges per item, one block each) and
 * grid cell size (one cell covering the roadmap, or 1, 2, 4 or 8 times the
 * mean edge extent), and one cell with items sized so that their count fills
 * 1, 2 or 3 rounds of the item blocks the device holds at once.  For each, the grid is rebuilt on the device and the updates
 * a -> b_i -> a for i = 0..n_b-1 are run `reps` times (0 selects 5) after one
 * untimed pass, timed with HIP events on the roadmap's own stream; the
 * fastest configuration is kept (the current one unless another is at least
 * 3% faster).  Labels never depend on the choice: every candidate must
 * reproduce the first candidate's gray counts, otherwise RGG_E_DEVICE.
 *
 * obstacles_a (m slots) must equal the resident obstacle slots, so the
 * roadmap's state is the same before and after (its counters return to their
 * values after each round trip); obstacles_b holds n_b (1..64) representative
 * next obstacle sets of m slots each, one after the other.  Host arrays.  The
 * call blocks.  It is refused with RGG_E_BUSY while a graph, a batch or a
 * server request holds the roadmap (their kernels hold its grid arrays);
 * RGG_E_STATE_MISMATCH if obstacles_a is not the resident state (nothing
 * changes); RGG_E_INVALID_ARG for bad arguments or a state b_i with an
 * invalid box; RGG_E_OUT_OF_MEMORY when a candidate grid does not fit.  After
 * an error the roadmap's state and labels are unchanged, its grid may be any
 * of the candidates.  *report (may be null) receives the choice and every
 * candidate's mean time per update. */
#define RGG_TUNE_MAX_CANDIDATES 32
typedef struct {
    int32_t n_candidates;
    int32_t item_edges;                               /* chosen                         */
    double cell_size;                                 /* chosen; +inf = one cell.
                                                         rgg_batch_tune: the factor of
                                                         each roadmap's mean edge extent */
    int64_t grid_cells[3];                            /* rgg_tune only                  */
    double us_per_update;                             /* chosen configuration           */
    double us_before;                                 /* the configuration before tuning */
    int32_t cand_item_edges[RGG_TUNE_MAX_CANDIDATES]; /* candidate 0 = before tuning
                                                         (rgg_batch_tune: 0, each
                                                         roadmap's own)                 */
    double cand_cell_size[RGG_TUNE_MAX_CANDIDATES];   /* +inf = one cell; rgg_batch_tune:
                                                         factor (0 = each roadmap's own) */
    double cand_us[RGG_TUNE_MAX_CANDIDATES];
} rgg_tune_report;
rgg_status rgg_tune(rgg_roadmap *rm, int64_t m, const rgg_box *obstacles_a, int32_t n_b,
                    const rgg_box *obstacles_b, int32_t reps, rgg_tune_report *report);

/* The autotuner for a batch: one work decomposition for all of the batch's
 * roadmaps (the same candidates as rgg_tune, the cell size as a factor of
 * each roadmap's own mean edge extent), timed on whole batched updates (the
 * batch's stage kernels over every roadmap, as rgg_batch_launch runs them):
 * roadmap k (in the batch's order) goes from obstacles_a[k] to
 * obstacles_b[k] and back, both host arrays of its own slot count, and
 * obstacles_a[k] must be its resident state.  us_per_update is the time of
 * one batched update.  The batch's previous launches are waited for; the
 * captured graph is rebuilt for the chosen decomposition.  RGG_E_BUSY if
 * another graph, batch or server request also holds one of the roadmaps.
 * Other errors as for rgg_tune. */
rgg_status rgg_batch_tune(rgg_batch *b, const rgg_box *const *obstacles_a, const rgg_box *const *obstacles_b,
                          int32_t reps, rgg_tune_report *report);

/* Full validation (Alg. 1 when not lazy: every edge left unknown gets a
 * full collision check).  Decides, for each listed edge, whether any
 * configuration q(t), t in [0, 1], of its motion puts a robot sphere into a
 * present obstacle slot, by refining the outer and inner approximations of
 * Sec. 3.2 on dyadic sub-intervals [j 2^-l, (j+1) 2^-l]: an interval is
 * free when every sphere's capsule between its centres at the interval's
 * ends, inflated to r_i + delta_i 4^-l, misses every box; the search tests
 * the robot at the midpoints of the intervals that are not free, level by
 * level, and splits them.
 *   verdict RGG_VERDICT_COLLIDES: witness[i] is the colliding parameter
 *     (0 or 1 first, else the smallest colliding midpoint of the first level
 *     with one); RGG_VERDICT_FREE: no configuration collides;
 *     RGG_VERDICT_UNRESOLVED: more than max_active intervals stayed unknown
 *     at some level, or max_level levels were not enough (a caller treats
 *     the edge as invalid); witness[i] is NaN unless COLLIDES; level[i] is
 *     the level where the search stopped.
 * Configurations use the binary64 motion of the build with a sin/cos made of
 * fixed binary64 steps, so verdicts are reproducible bit for bit.  The
 * obstacles are the roadmap's resident slots when the validation runs (after
 * its queued updates).  max_level 0..30 (0: RGG_VALIDATE_DEFAULT_LEVELS),
 * max_active 1..512 (0: RGG_VALIDATE_DEFAULT_ACTIVE).
 * rgg_validate: host arrays ids[n] (each an edge id, else RGG_E_INVALID_ARG),
 * verdict[n], level[n] and witness[n] (level and witness may be NULL);
 * returns when done.
 * rgg_validate_async: device arrays (d_verdict, d_level and d_witness may
 * each be NULL when d_labels is given), queued on `stream` after the
 * roadmap's previous update.  When d_count is non-null (the result of an update queued
 * before, e.g. with d_ids its gray list), only the first
 * min(n, d_count->n_gray) ids are validated, and none if that update failed;
 * an id that is not an edge gets RGG_VERDICT_BAD_ID.  Entries past the
 * validated count are left as they were.  When d_labels (a device label
 * array of the roadmap's E edges, e.g. the update's) is non-null, each
 * validated edge's label becomes RGG_GREEN (FREE) or RGG_RED (COLLIDES or
 * UNRESOLVED): after rgg_update_async and this call on one stream it holds
 * the non-lazy labels, with no GRAY left among the validated edges.  The
 * roadmap's own state (its counters, rgg_labels) keeps the RGG labels. */
#define RGG_VALIDATE_DEFAULT_LEVELS 24
#define RGG_VALIDATE_DEFAULT_ACTIVE 256
rgg_status rgg_validate(rgg_roadmap *rm, const int64_t *ids, int64_t n, int32_t max_level, int32_t max_active,
                        uint8_t *verdict, int32_t *level, double *witness);
rgg_status rgg_validate_async(rgg_roadmap *rm, void *stream, const int64_t *d_ids, int64_t n,
                              const rgg_update_result *d_count, int32_t max_level, int32_t max_active,
                              uint8_t *d_verdict, int32_t *d_level, double *d_witness, uint8_t *d_labels);

/* Persistence between planning iterations (Sec. 1 and Sec. 4.3: the
 * approximations are computed once and then stored and reloaded).
 * rgg_save writes `rm` to the file `path`: its binary64 sphere centres and
 * capsules, edge boxes, sphere radii, the resident obstacle slots, the per-edge
 * counters, the precision mode, band, re-test capacity and the work
 * decomposition (cell size, edges per item), the robot and the edges'
 * motions for rgg_validate, followed by an FNV-1a 64-bit checksum; host byte
 * order, format version 2.  It first waits for the
 * roadmap's queued updates.  RGG_E_BUSY if a graph, batch or server request
 * holds the roadmap; RGG_E_INVALID_ARG if the file cannot be written.
 * rgg_load builds a roadmap on ctx's device from such a file without
 * recomputing the kinematics: its labels, gray list and every later update
 * equal those of the saved roadmap.  RGG_E_INVALID_ARG if the file cannot be
 * read, is not a roadmap file, has another version, an inconsistent header,
 * is truncated or fails the checksum; RGG_E_OUT_OF_MEMORY, RGG_E_DEVICE.
 * *out receives the roadmap (destroy it with rgg_destroy). */
rgg_status rgg_save(rgg_roadmap *rm, const char *path);
rgg_status rgg_load(rgg_context *ctx, const char *path, rgg_roadmap **out);

/* Request server (continuous batching).  A worker thread takes the queued
 * updates of device-resident roadmaps to the GPU as batches (one launch per
 * stage for the whole batch, as rgg_batch_launch), on n_streams streams, so
 * requests that arrive while others run are admitted into the next batch
 * and their work overlaps on the device.  Admission is by memory: each
 * request's obstacle boxes are staged in a device pool of pool_bytes, and a
 * request is dispatched only when its 2*m boxes fit in the pool's free space
 * (requests of one roadmap keep their submission order; the next one may
 * start before the previous one has finished, ordered on the device).  Each
 * request computes exactly what rgg_update_async computes for it. */
typedef struct rgg_server rgg_server;

typedef struct {
    int32_t n_streams;            /* batches in flight at once; 0 = 4, max 16   */
    int32_t max_queue;            /* queued requests; 0 = 4096                  */
    int32_t max_batch;            /* requests per batch; 0 = 64, max 256        */
    int32_t reserved;             /* must be 0                                  */
    int64_t pool_bytes;           /* device staging for the requests' boxes, the
                                     memory that admits requests (a request waits
                                     until its boxes fit); 0 = admission by free
                                     device memory: 1/64 of the memory free when
                                     the server starts, within [16 MiB, 256 MiB].
                                     A value above the free memory is refused   */
} rgg_server_opts;

typedef struct {
    rgg_roadmap *rm;              /* resident roadmap; not updated elsewhere
                                     while the server holds requests for it     */
    int64_t m;                    /* = its n_obstacle_slots                     */
    const rgg_box *old_boxes;     /* [m] host; copied by rgg_server_submit      */
    const rgg_box *new_boxes;     /* [m] host; copied by rgg_server_submit      */
    uint8_t *d_labels;            /* [E] device or NULL; written in order       */
    int64_t *d_gray;              /* [gray_cap] device or NULL                  */
    int64_t gray_cap;
    int32_t validate;             /* non-zero: non-lazy (Alg. 1 when not lazy):
                                     after the update, the gray list is validated
                                     as rgg_validate_async with default limits and
                                     d_labels / d_gray (both required) given, so
                                     d_labels ends with GREEN or RED for every
                                     validated gray edge                        */
    uint8_t *d_verdict;           /* [gray_cap] device or NULL: the verdicts of
                                     the validated gray list entries            */
} rgg_server_req;

/* Starts the server (its worker thread and streams) on ctx's device. */
rgg_status rgg_server_start(rgg_context *ctx, const rgg_server_opts *opts, rgg_server **out);
/* Queues one update; *ticket identifies it.  RGG_E_BUSY if the queue is
 * full, RGG_E_INVALID_ARG for a malformed request or one whose boxes can
 * never fit the pool.  The boxes are copied before it returns. */
rgg_status rgg_server_submit(rgg_server *srv, const rgg_server_req *req, uint64_t *ticket);
/* State of a ticket: *done = 0 (queued or running) or 1 (finished; *result
 * and *latency_us, submission to completion, are set and the ticket is
 * released).  wait != 0 blocks until it has finished.  RGG_E_INVALID_ARG for
 * an unknown ticket. */
rgg_status rgg_server_poll(rgg_server *srv, uint64_t ticket, int32_t wait, int32_t *done,
                           rgg_update_result *result, double *latency_us);

/* Where a request's time went (host clock, microseconds). */
typedef struct {
    double latency_us;            /* submission to completion                   */
    double queue_us;              /* submission to its batch's launch: waiting
                                     for a free stream slot, pool room or the
                                     roadmap's earlier request                  */
    double service_us;            /* launch to completion: the batch's copies and
                                     kernels on the device (with the roadmaps'
                                     earlier updates it waits for) and the
                                     worker noticing the finish                 */
    int32_t batch_size;           /* requests in its batch                      */
    int32_t reserved;
} rgg_request_timing;

/* rgg_server_poll with the request's time split into queue and service. */
rgg_status rgg_server_poll_timing(rgg_server *srv, uint64_t ticket, int32_t wait, int32_t *done,
                                  rgg_update_result *result, rgg_request_timing *timing);
/* The server's effective options (the pool size chosen when pool_bytes was
 * 0) and the free device memory it saw when it started. */
rgg_status rgg_server_info(rgg_server *srv, rgg_server_opts *opts, int64_t *free_at_start);
/* Finishes every queued request, then stops the worker and frees the server. */
rgg_status rgg_server_stop(rgg_server *srv);

/* Current labels [E] / gray list of the last update, copied to host memory.
 * rgg_gray_list writes min(n, cap) ids and sets *n to the full count. */
rgg_status rgg_labels(rgg_roadmap *rm, uint8_t *out);
rgg_status rgg_gray_list(rgg_roadmap *rm, int64_t *out, int64_t cap, int64_t *n);

/* Per-update kernel timing with HIP events on the update's stream (off by
 * default).  rgg_timing_read returns the summed milliseconds of each stage
 * over the updates since the last read, and resets them:
 * ms[0] diff, ms[1] grid cells, ms[2] the FP32 item kernel (pair listing
 * and the inline pair tests: every test by default), ms[3] the balanced pair
 * testing (FP32 mode with pair listing) or the binary64 item kernel (FP64
 * mode), ms[4] FP64 re-test, ms[5] labels and gray compaction.  *n_updates
 * receives the number of updates timed.  Each event adds a few microseconds
 * to the timeline of a timed update. */
rgg_status rgg_timing_enable(rgg_roadmap *rm, int32_t on);
rgg_status rgg_timing_read(rgg_roadmap *rm, double ms[6], int64_t *n_updates);

/* Host-only view of the build stage, for tests: computes the approximations
 * of edge range [e0, e1) exactly as rgg_build does, without any device.
 * n_configs [e1-e0] receives |cfg(e)|; centres [sum |cfg(e)|][B][D] the
 * sphere centres; capsule [e1-e0][B][2D+1] (A, B, R); aabb [e1-e0][6] the
 * padded FP32 edge box (lo, hi).  Pass NULL centres/capsule/aabb to query
 * n_configs only. */
rgg_status rgg_debug_geometry(const rgg_roadmap_desc *roadmap, const rgg_robot *robot,
                              const rgg_build_opts *opts, int64_t e0, int64_t e1,
                              int64_t *n_configs, double *centres, double *capsule,
                              float *aabb);

/* Host-only view of the second forms (opts->outer_obb, opts->inner_splines)
 * of edge range [e0, e1), computed exactly as rgg_build does, for tests.
 * obb [e1-e0][bodies][2D + D*D] (centre, axes as rows, half-extents; zero
 * for a body without spheres; bodies = 1, or n_links for the arm) when
 * opts->outer_obb; n_segments [(e1-e0) * B] the spline segments kept for
 * each (edge, sphere) and segments [sum][2D+1] (A, B, rho) when
 * opts->inner_splines.  Any output may be NULL (query n_segments first to
 * size segments). */
rgg_status rgg_debug_second_forms(const rgg_roadmap_desc *roadmap, const rgg_robot *robot,
                                  const rgg_build_opts *opts, int64_t e0, int64_t e1, double *obb,
                                  int64_t *n_segments, double *segments);

/* Host-only view of rgg_load, for tests: reads the roadmap file `path` and
 * runs every check rgg_load runs before it uses the device (header, sample
 * offsets with 2 .. 2^24 configurations per edge, robot, truncation,
 * checksum); *n_edges (may be NULL) receives its edge count.  Same errors as
 * rgg_load's file checks. */
rgg_status rgg_debug_read_file(const char *path, int64_t *n_edges);

const char *rgg_last_error(void);
const char *rgg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RGG_H */
