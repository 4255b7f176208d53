/*
 * mf.h -- exact s-t minimum cut / maximum flow on grid graphs by parallel
 * augmented-path region discharge (P-ARD), on one AMD Instinct MI355X (gfx950).
 *
 * Problem (paper Sec. 2, eq. (1)): a network G = (V, E, s, t, c, e) with
 * integer capacities.  Here V is a 2D or 3D grid, E joins each vertex to its
 * grid neighbours at the canonical offsets below, c(s, v) and c(v, t) are the
 * terminal links.  The library computes a maximum preflow (Sec. 2: no vertex
 * with positive excess reaches t in the residual network), its flow value
 * |f| = sum_v f(v, t), and the two extremal minimum cuts.
 *
 * Method: the grid is partitioned into box regions (Sec. 3, fixed partition);
 * each sweep discharges every region holding an active vertex against the
 * boundary labels of the previous sweep (Alg. 2), where a discharge moves
 * excess to t first and then to boundary vertices in increasing label order
 * and finally relabels the region (Proc. ARD, Sec. 4.2; region relabel,
 * Alg. 3); flows over boundary arcs are then fused under the valid-pair rule
 * of Alg. 2 and the global gap heuristic over boundary labels is applied
 * (Sec. 5.1).  Sweeps repeat until no vertex is active (Sec. 4.4).
 *
 * Everything runs in HIP kernels on the device; there is no CPU fallback.
 *
 * Conventions shared by every entry point
 *   - dims are row-major, last axis fastest: 2D {H, W}, 3D {D, H, W}; vertex
 *     v has index y*W + x (2D) or (z*H + y)*W + x (3D).
 *   - connectivity 4 or 8 (2D) or 6 (3D); canonical offsets, opposite
 *     directions adjacent (reverse of direction k is k ^ 1):
 *       2D-4: +x, -x, +y, -y
 *       2D-8: 2D-4 then +x+y, -x-y, +x-y, -x+y
 *       3D-6: +x, -x, +y, -y, +z, -z
 *   - capacities are int32 >= 0; the flow value is int64.
 *   - status codes: no entry point throws; every failure is reported by the
 *     returned mf_status and leaves the handle usable unless MF_E_DEVICE.
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mf_grid mf_grid; /* opaque, owned by the library */

typedef enum {
    MF_OK = 0,
    MF_E_INVAL = 1,    /* bad argument: shape, connectivity, negative or out-of-grid capacity */
    MF_E_NOMEM = 2,    /* device or host allocation failed */
    MF_E_DEVICE = 3,   /* a HIP call failed or a kernel reported an internal error */
    MF_E_STATE = 4,    /* call order violated (e.g. solve before set_caps) */
    MF_E_OVERFLOW = 5, /* capacities could overflow int32 residuals or excesses */
    MF_E_SWEEPS = 6    /* max_sweeps reached before the preflow became maximum */
} mf_status;

/* which minimum cut mf_min_cut returns */
enum {
    MF_CUT_MIN_SOURCE = 0, /* unique minimal source side: s and every vertex an
                              excess vertex reaches in the final residual network */
    MF_CUT_MAX_SOURCE = 1  /* the paper's (T-bar, T): every vertex that does not reach t */
};

/* region schedule inside a sweep */
enum {
    MF_SCHED_PARD = 0,    /* Alg. 2: all active regions against the previous sweep's labels */
    MF_SCHED_COLORED = 1, /* Alg. 1 as phases of non-interacting regions: one colour class
                             (2 for 4- and 6-connected grids, 4 for 2D 8-connected) per
                             phase, its flow and labels applied before the next phase; a
                             sweep is one phase per colour.  Not with boundary_relabel or
                             features (MF_E_INVAL) */
    MF_SCHED_LEARNED = 2, /* deferral from a trained scorer (opts->model); the regions to
                             discharge are queued longest previous discharge first; at most
                             65536 regions, else MF_E_INVAL */
    MF_SCHED_AUTO = 3,    /* library's choice (currently MF_SCHED_PARD) */
    MF_SCHED_LEARNED_COLORED = 4 /* the learned scheduler driving the colour phases of
                             MF_SCHED_COLORED: at the start of each sweep the network scores
                             the regions, the phases run in descending order of the predicted
                             progress summed over each colour's active regions, and the
                             deferral rule of MF_SCHED_LEARNED applies inside a phase */
};

typedef struct {
    int32_t schedule;             /* MF_SCHED_*; 0 is P-ARD */
    int32_t global_relabel_every; /* exact region-distance relabel every N sweeps; 0 = off */
    int32_t gap;                  /* 1 = global gap heuristic on (default), 0 = off */
    int32_t check_every;          /* sweeps enqueued between host-side termination checks; 0 = 8 */
    int64_t max_sweeps;           /* guard; 0 = 2|B|^2 + 1 (the bound of Sec. 4.3-4.4), at least
                                   * 2^20 with round_cap > 0, where that bound does not hold */
    const void *model;            /* mf_model * for MF_SCHED_LEARNED, else NULL */
    void *stream;                 /* hipStream_t to run on; NULL = the null stream */
    int32_t profile;              /* 1 = time every discharge launch with HIP events */
    int32_t region_kernel;        /* MF_KERNEL_*: where a discharging region lives */
    int32_t *trace;               /* device buffer of MF_TRACE_FIELDS x trace_cap int32, or NULL:
                                     one record per region discharge, see MF_TR_* */
    int64_t trace_cap;            /* records the trace buffer holds; extra records are dropped */
    int32_t graph;                /* 1 = replay batches of sweeps as a captured HIP graph (ignored
                                     with profile, trace, features or MF_SCHED_LEARNED); a NULL
                                     stream is then replaced by a stream owned by the handle */
    int32_t max_defer;            /* MF_SCHED_LEARNED: consecutive deferrals after which a region
                                     is discharged anyway; 0 = 2 */
    float defer_threshold;        /* MF_SCHED_LEARNED: defer an active region whose predicted
                                     probability of useful work is below this; 0 = 0.5 */
    int32_t defer_mode;           /* MF_SCHED_LEARNED: 0 = a deferred region is skipped (labels carried
                                     over); 1 = it only runs its region relabel (Alg. 3 on the current
                                     state, no pushes) */
    float *features;              /* device buffer [features_cap][regions][MF_FEATURES] or NULL:
                                     the scheduler's region features at the start of each sweep */
    int64_t features_cap;         /* sweeps the features buffer holds */
    int32_t partial;              /* 1 = partial discharges (Sec. 6.2): in sweep s a region discharge
                                     runs only the stages k <= s of Proc. ARD (sweep 0 augments to
                                     t only), the region relabel stays complete, and excess the cap
                                     holds back stays active for later sweeps; the flow and cuts are
                                     the same, sweeps can be more and cheaper.  0 = off */
    int32_t boundary_relabel;     /* n in 1..4096: the boundary relabel heuristic (Sec. 6.1, see
                                     mf_boundary_relabel) after the flow fusion of every sweep,
                                     before the gap, with at most n levels of its search per sweep
                                     (labels it has not reached by then are lifted to n + 1 at most,
                                     which keeps them valid); n level kernels are launched per sweep
                                     (those after the search ended exit at once).  0 = off */
    int32_t method;               /* MF_METHOD_ARD (0): augmented-path region discharge (Sec. 4);
                                     MF_METHOD_PRD (1): push-relabel region discharge (Sec. 3,
                                     Proc. PRD) under the same parallel driver (Alg. 2), with the
                                     distance labels of Sec. 2 (every arc counts, d_inf = n), the
                                     global gap over all labels and the HBM region kernel; not
                                     combined with partial, boundary_relabel, global_relabel_every,
                                     features or MF_SCHED_LEARNED (MF_E_INVAL) */
    int32_t *label_trace;         /* device buffer [label_trace_cap][n] int32, or NULL: the labels
                                     (row-major like dims) after every step, a sweep of Alg. 2 or a
                                     colour phase of Alg. 1, after its fusion and gap; steps beyond
                                     label_trace_cap are not recorded.  Forces eager launches (no
                                     graph) */
    int64_t label_trace_cap;      /* steps the label trace holds */
    int32_t round_cap;            /* n >= 1: a region discharge runs at most n search-and-push rounds
                                     per sweep; excess its last (complete, label-writing) search still
                                     finds reaching a target stays in the region, which stays active
                                     for the next sweep (the mechanism of partial discharges, Sec. 6.2,
                                     with a cap on rounds instead of stages).  A sweep lasts as long
                                     as its slowest region: the cap shortens the longest discharges
                                     and lets the others go on in the next sweep.  The flow and cuts
                                     are the same.  0 = off; not with MF_METHOD_PRD (MF_E_INVAL) */
} mf_solve_opts;

/* region discharge operation, see mf_solve_opts.method */
enum { MF_METHOD_ARD = 0, MF_METHOD_PRD = 1 };

/* region features (floats) written per region and sweep, see mf_solve_opts.features */
enum {
    MF_FT_EXCESS = 0,     /* log1p(total excess of active vertices) / 8 */
    MF_FT_LABEL = 1,      /* log1p(mean finite label of the region's border vertices) / 8 */
    MF_FT_RESDEG = 2,     /* fraction of outgoing boundary arcs with positive residual */
    MF_FT_ACTIVE = 3,     /* 1 if the region holds an active vertex */
    MF_FT_LABEL_SUM = 4,  /* sum over border vertices of min(label, 65535) */
    MF_FT_EXCESS_RAW = 5, /* total excess of active vertices */
    MF_FEATURES = 6
};

/* trace record fields (int32 each) */
enum {
    MF_TR_SWEEP = 0,      /* sweep index, from 0 */
    MF_TR_REGION = 1,     /* region id (z-major over the region grid) */
    MF_TR_ROUNDS = 2,     /* search + push rounds of the discharge */
    MF_TR_LEVELS = 3,     /* breadth-first search levels over all rounds */
    MF_TR_STAGES = 4,     /* boundary stages opened over all rounds */
    MF_TR_TICKS = 5,      /* duration in ticks of the 100 MHz device wall clock */
    MF_TR_EXCESS_IN = 6,  /* total excess of the region when the discharge started (saturated) */
    MF_TR_TO_SINK = 7,    /* flow the discharge sent to t */
    MF_TR_TO_BOUNDARY = 8,/* flow the discharge pushed over boundary arcs */
    MF_TR_LABEL_SUM = 9,  /* sum over the region's boundary vertices of min(new label, 65535) */
    MF_TRACE_FIELDS = 10
};

/* region_kernel values */
enum {
    MF_KERNEL_AUTO = 0, /* WAVE for 2D regions up to 64 x 64, else ROWS or ROWS64 when
                           applicable, else LDS when it fits, else HBM */
    MF_KERNEL_HBM = 1,  /* region state stays in HBM; search arrays in LDS or HBM scratch */
    MF_KERNEL_LDS = 2,  /* whole region in LDS, one workgroup; MF_E_INVAL if it does not fit */
    MF_KERNEL_WAVE = 3, /* 2D region of at most 64 x 64 in LDS, one wavefront, row-bitmask
                           search; MF_E_INVAL if not applicable */
    MF_KERNEL_ROWS = 4, /* 3D 6-connected region with rows of 32 along x, 2 <= ty, 2 <= tz,
                           ty * tz a multiple of 64 and at most 1024: one 1024-thread
                           workgroup, row-bitmask search and parallel pushes, state in HBM;
                           MF_E_INVAL if not applicable */
    MF_KERNEL_ROWS64 = 5 /* 3D 6-connected region with rows of 64 along x (64^3 regions), 2 <= ty,
                           2 <= tz, ty * tz a multiple of 64 and at most 4096: one 512-thread
                           workgroup with eight rows per thread in registers, row-bitmask
                           search, masks and admissible arcs in per-workgroup scratch, state
                           in HBM; MF_E_INVAL if not applicable */
};

typedef struct {
    int64_t sweeps;             /* sweeps that started with an active vertex (Sec. 3) */
    int64_t region_discharges;  /* regions discharged, summed over sweeps */
    int64_t boundary_size;      /* |B| (Sec. 4.1), geometric */
    int64_t d_inf;              /* max(|B|, 1) */
    double solve_ms;            /* wall time of mf_solve, host clock, stream synchronised */
    double discharge_ms;        /* profile=1: summed duration of the discharge launches */
    int64_t discharge_launches; /* profile=1: number of timed discharge launches */
    double discharge_bytes;     /* algorithmic bytes of all discharges, see mf_discharge_bytes_per_vertex */
    int64_t discharged_vertices;/* real vertices in discharged regions, summed over sweeps */
    int64_t discharge_iterations; /* search + push rounds, summed over all discharges */
    int64_t search_levels;      /* breadth-first search levels, summed over all searches */
    int64_t search_stages;      /* boundary stages opened by the searches (targets d(w)+1) */
    int64_t trace_records;      /* records written to opts->trace (may exceed trace_cap) */
    int64_t search_ticks;       /* 100 MHz device-clock ticks in searches, summed over workgroups */
    int64_t push_ticks;         /* 100 MHz device-clock ticks in push passes, summed over workgroups */
    int64_t setup_ticks;        /* part of search_ticks spent resetting and seeding a search */
    int64_t flood_ticks;        /* part of search_ticks spent in the in-region floods */
    int64_t global_relabels;    /* exact region-distance relabels performed */
    int64_t global_relabel_levels; /* distance levels over all global relabels */
    int64_t push_iterations;    /* parallel push iterations, summed over discharges */
    int64_t region_kernel;      /* MF_KERNEL_* that ran the region discharges */
    int64_t relabel_only;       /* deferred regions that ran their region relabel only (defer_mode 1) */
} mf_solve_stats;

/* Create a solver handle for a grid shape and region partition.
 *   ndim          2 or 3
 *   dims          [ndim] grid extents, each >= 1, product < 2^31
 *   connectivity  4 or 8 for ndim = 2, 6 for ndim = 3
 *   region_shape  [ndim] box region extents (Sec. 3 fixed partition; the last
 *                 region along an axis may be partial), or NULL / all zeros to
 *                 let the library pick
 *   out           receives the handle; unchanged on failure
 * Allocates all device memory for the shape.  Errors: MF_E_INVAL, MF_E_NOMEM,
 * MF_E_DEVICE.  Uses the current HIP device. */
mf_status mf_create_grid(int32_t ndim, const int64_t *dims, int32_t connectivity,
                         const int32_t *region_shape, mf_grid **out);

/* Load an instance (Sec. 2 network; Init of Sec. 2 happens in mf_solve).
 *   src_cap   [n]     c(s, v) >= 0
 *   sink_cap  [n]     c(v, t) >= 0
 *   nbr_cap   [K][n]  c(v, v + o_k) >= 0, 0 where v + o_k leaves the grid
 *   on_device 0: the three pointers are host memory; 1: device memory of the
 *             current device (e.g. torch CUDA tensors); the library copies
 *             them and keeps no reference.
 *   stream    hipStream_t used for the copies and checks, or NULL
 * Errors: MF_E_INVAL (negative capacity or non-zero capacity on an arc that
 * leaves the grid), MF_E_OVERFLOW (c(u,v) + c(v,u) > INT32_MAX, or
 * c(s,v) + sum_u c(u,v) > INT32_MAX), MF_E_DEVICE.  On error the handle holds
 * no instance (a following mf_solve returns MF_E_STATE). */
mf_status mf_set_caps(mf_grid *g, const int32_t *src_cap, const int32_t *sink_cap,
                      const int32_t *nbr_cap, int32_t on_device, void *stream);

/* Solve the loaded instance to a maximum preflow.  opts may be NULL
 * (defaults: P-ARD, gap on, global relabel off).  st may be NULL.  Blocks
 * until the result is on the device and the stream is synchronised.  A second
 * call re-solves the same instance from Init.  st is filled on MF_OK and on
 * MF_E_SWEEPS (then with the sweeps run up to the limit).
 * Errors: MF_E_STATE (no instance), MF_E_SWEEPS, MF_E_DEVICE, MF_E_INVAL. */
mf_status mf_solve(mf_grid *g, const mf_solve_opts *opts, mf_solve_stats *st);

/* Flow value |f| = sum_v (c(v,t) - c_f(v,t)) of the last solve (Sec. 2).
 * Errors: MF_E_STATE if no solve has completed. */
mf_status mf_flow_value(const mf_grid *g, int64_t *out);

/* Minimum cut of the last solve as a source-side indicator.
 *   kind             MF_CUT_MIN_SOURCE or MF_CUT_MAX_SOURCE
 *   out_source_side  [n] host array, 1 = source side, row-major like dims
 * Computed on the device by residual reachability.  Errors: MF_E_STATE,
 * MF_E_INVAL, MF_E_DEVICE. */
mf_status mf_min_cut(const mf_grid *g, int32_t kind, uint8_t *out_source_side);

/* State after the last solve (completed, or stopped by max_sweeps with
 * MF_E_SWEEPS) in the row-major layout of the inputs, for certification:
 * residuals [K][n] (c_f(v, v+o_k)), residual t-links [n], excess [n], labels
 * [n].  Any pointer may be NULL.  Host arrays.  Errors: MF_E_STATE if no solve
 * has left a state, MF_E_DEVICE. */
mf_status mf_get_state(const mf_grid *g, int32_t *res, int32_t *rt, int32_t *ex, int32_t *labels);

/* Boundary relabel heuristic (Sec. 6.1) on the state the last solve left
 * (see mf_get_state).  The labels of the boundary vertices B with d(u) < dinf
 * are grouped by region and label; a group reaches the group of the next larger
 * label of its region at length 0, and the group of u reaches the group of w at
 * length 1 for every residual arc (u, w) between regions.  d'(u) is the distance
 * from u's group to a group of label 0 and the labels of B become
 * max(d(u), min(d'(u), dinf)); interior labels are left as they are (the next
 * discharge of a region recomputes them before anything reads them).
 *   max_levels  n > 0: at most n levels of the search (unreached labels are
 *               lifted to n + 1 at most, a valid lower bound)
 *   levels_out  receives the number of levels that assigned a distance (may be NULL)
 * Runs on the device (one workgroup per region and level, levels launched in
 * batches of eight until the search ends).  Errors: MF_E_INVAL, MF_E_STATE
 * (also for a state left by MF_METHOD_PRD, whose labels are not region
 * distances), MF_E_DEVICE. */
mf_status mf_boundary_relabel(mf_grid *g, int32_t max_levels, int64_t *levels_out);

/* Region relabel (Alg. 3, the ARD variant of Sec. 4.2) of every region on the
 * state the last solve left (see mf_get_state), as the last search of a region
 * discharge computes it, without pushes: for u in region R, d(u) = 0 if u
 * reaches t in the region network G^R, else 1 + min d(w) over the boundary
 * vertices w with d(w) < dinf that u reaches through a residual boundary arc,
 * else dinf, with the current labels as d(w).  Every label of the state is
 * replaced (border vertices included); residuals, t-links and excess stay.
 *   region_kernel  MF_KERNEL_* that runs it (AUTO as for mf_solve)
 *   regions_out    receives the number of regions relabelled (may be NULL)
 * Errors: MF_E_STATE (no state, or a state left by MF_METHOD_PRD), MF_E_INVAL
 * (kernel not applicable), MF_E_NOMEM, MF_E_DEVICE. */
mf_status mf_region_relabel(mf_grid *g, int32_t region_kernel, int64_t *regions_out);

/* Exact region-distance relabel (Sec. 4.1) on the state the last solve left:
 * every label becomes min(d*B(u), dinf), d*B the distance to t in the residual
 * network where an arc between regions has length 1 and an arc inside a region
 * length 0 (a 0-1 breadth-first search backwards from the vertices with a
 * residual t-link, one launch per distance level).
 *   levels_out  receives the number of level launches (a multiple of four; may be NULL)
 * Errors: MF_E_STATE (no state, or a state left by MF_METHOD_PRD), MF_E_DEVICE. */
mf_status mf_global_relabel(mf_grid *g, int64_t *levels_out);

/* Region reduction (Alg. 5, Sec. 8) of every region of the loaded instance: one
 * class byte per vertex (row-major like dims), the OR of
 *   MF_REDUCE_STRONG_SOURCE  in the source side of every minimum cut
 *   MF_REDUCE_STRONG_SINK    in the sink side of every minimum cut
 *   MF_REDUCE_WEAK_SOURCE    in the source side of some minimum cut
 *   MF_REDUCE_WEAK_SINK      in the sink side of some minimum cut
 * as Alg. 5 decides them from the region network alone (R, its boundary B^R
 * without s- and t-links, the arcs touching R); a vertex none of them marks is
 * undecided.  Alg. 5's single flow gives the classes of the two auxiliary
 * problems the section starts from, each boundary vertex joined to t without
 * bound (strong source = its minimal source side, weak source = its maximal
 * minus its minimal source side) or supplied from s without bound (strong
 * sink = outside its maximal source side, weak sink = its maximal minus its
 * minimal source side); they are computed that way, for all regions at once:
 * Init, a full discharge of every region with the boundary labels 0 (every
 * residual boundary arc a target) or dinf after saturating every arc into the
 * region, and a forward search from the remaining excess inside each region.
 *   region_kernel  MF_KERNEL_* that runs the discharges (AUTO as for mf_solve)
 *   out_class      [n] host array
 * Overwrites the solver state (call mf_solve again before mf_flow_value,
 * mf_min_cut or mf_get_state).  Errors: MF_E_STATE (no instance loaded),
 * MF_E_INVAL (batch handle, kernel not applicable), MF_E_DEVICE. */
enum {
    MF_REDUCE_STRONG_SOURCE = 1,
    MF_REDUCE_STRONG_SINK = 2,
    MF_REDUCE_WEAK_SOURCE = 4,
    MF_REDUCE_WEAK_SINK = 8
};
mf_status mf_region_reduction(mf_grid *g, int32_t region_kernel, uint8_t *out_class);

/* Shape facts of a handle: number of vertices, K, regions, |B|, region shape. */
mf_status mf_get_info(const mf_grid *g, int64_t *n, int32_t *K, int64_t *regions,
                      int64_t *boundary_size, int32_t *region_shape3);

/* ---- Batches: many independent 2D instances solved together (one sweep
 * launch discharges regions of every instance from one work queue).  The
 * instances are packed, region-aligned, on one canvas with no arcs between
 * them, so the canvas maximum flow is the union of the instance maximum flows
 * (Sec. 2 network of each instance unchanged); a 4-connected instance is
 * carried with zero diagonal capacities when the batch holds 8-connected ones.
 *
 * mf_create_batch
 *   count         number of instances (>= 1)
 *   dims          [count][2] row-major {H, W} of each instance
 *   connectivity  [count] 4 or 8
 *   region_shape  [2] region extents shared by all instances, or NULL / zeros
 *                 for 32 x 32
 * The handle works with mf_solve, mf_flow_value (sum over instances),
 * mf_destroy and the mf_batch_* calls below; mf_set_caps on it is MF_E_INVAL. */
mf_status mf_create_batch(int32_t count, const int64_t *dims, const int32_t *connectivity,
                          const int32_t *region_shape, mf_grid **out);

/* Placement of instance `index` on the canvas (offset {y, x} and dims {H, W}),
 * or with index = -1 the canvas itself (offset {0, 0}). */
mf_status mf_batch_info(const mf_grid *g, int32_t index, int64_t *canvas_offset2,
                        int64_t *canvas_dims2);

/* Load instance `index` (same layout, rules and errors as mf_set_caps, with
 * that instance's dims and connectivity).  mf_solve needs every instance loaded
 * (MF_E_STATE otherwise). */
mf_status mf_batch_set_caps(mf_grid *g, int32_t index, const int32_t *src_cap,
                            const int32_t *sink_cap, const int32_t *nbr_cap, int32_t on_device,
                            void *stream);

/* Flow value of every instance after mf_solve: out[count] (int64). */
mf_status mf_batch_flow_values(const mf_grid *g, int64_t *out);

/* Minimum cut of instance `index` (kind as for mf_min_cut), out[H*W] host. */
mf_status mf_batch_min_cut(const mf_grid *g, int32_t index, int32_t kind, uint8_t *out_source_side);

/* ---- Learned region scheduler: a CNN over the grid of regions (channels
 * last, region id order: z-major, x fastest) with 3 input channels (the first
 * three region features), two hidden layers of `channels` ReLU units and one
 * output logit per region, all 3x3x3 convolutions with zero padding.  Trained
 * here with FP32 forward/backward kernels and Adam; used by MF_SCHED_LEARNED
 * in BF16 (weights and activations rounded to bfloat16, FP32 accumulation).
 * The score only orders and defers discharges; it never changes the result. */
typedef struct mf_model mf_model;

/* New model with He-uniform weights from `seed` and zero biases. */
mf_status mf_model_create(int32_t channels, uint64_t seed, mf_model **out);
void mf_model_destroy(mf_model *m);
/* Number of parameters: w1[C][3][27] b1[C] w2[C][C][27] b2[C] w3[1][C][27] b3[1]. */
int64_t mf_model_num_params(const mf_model *m);
mf_status mf_model_get_params(const mf_model *m, float *host_out);
mf_status mf_model_set_params(mf_model *m, const float *host_in);
/* logits[v] for a D x H x W grid of feature vectors x (device, stride xs floats
 * per voxel, channels 0..2 used); bf16 = 1 for the inference precision. */
mf_status mf_model_forward(mf_model *m, const float *x, int32_t xs, int32_t D, int32_t H, int32_t W,
                           float *logits, int32_t bf16, void *stream);
/* FP32 forward, binary cross-entropy with logits averaged over mask[v] = 1
 * voxels (target, mask device arrays [D*H*W]), backward into the model's
 * gradient buffer; loss and (if not NULL) the gradients are copied to host. */
mf_status mf_model_loss_grad(mf_model *m, const float *x, int32_t xs, const float *target,
                             const float *mask, int32_t D, int32_t H, int32_t W, float *loss,
                             float *grads_out, void *stream);
/* mf_model_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result, with the hidden activations in a fixed 4 MiB device
 * array of the library (one per GPU, kept until the process ends) instead of
 * the model's workspace.  Allocates nothing.  Limit: 2 * channels * D * H * W
 * <= 2^20 floats (32768 voxels with 16 channels), else MF_E_INVAL.  Every call
 * on a GPU uses that GPU's array: calls that overlap on one GPU (other host
 * threads, or other streams) race and must not run concurrently.
 * Errors: MF_E_INVAL, MF_E_DEVICE. */
mf_status mf_model_forward_noalloc(const mf_model *m, const float *x, int32_t xs, int32_t D, int32_t H,
                                   int32_t W, float *logits, int32_t bf16, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradients. */
mf_status mf_model_adam_step(mf_model *m, float lr, void *stream);

/* Algorithmic bytes one discharged vertex moves: its K residuals, residual
 * t-link and excess are read and written, its label is written. */
int64_t mf_discharge_bytes_per_vertex(int32_t connectivity);

/* ------------------------------------------------------------------------
 * General networks in region pages (Sec. 5.3).
 *
 * Any network given as vertex pairs, with any partition into regions, solved
 * by the same parallel region discharge (Alg. 2 with Proc. ARD, the region
 * relabel of Alg. 3, the flow fusion of Alg. 2 and the global gap of Sec. 5.1).
 * The splitter of Sec. 5.3 (host code inside mf_create_graph) numbers the
 * vertices region by region and writes one page per region: the region's arcs
 * with 32-bit offsets inside the page and its part of the preflow state.
 * Pairs between two regions stay in a resident boundary table of
 * O(|B| + |(B, B)|) words.  The pages either all live in HBM or are streamed:
 * they stay in pinned host memory and pass through device_pages page slots,
 * the next batch loaded while the current one is discharged (the streaming
 * mode of Sec. 5.3, with host memory in the role of the disk).
 * ------------------------------------------------------------------------ */
typedef struct mf_graph mf_graph; /* opaque, owned by the library */

typedef struct {
    int64_t n, npairs;           /* vertices and pairs of the network */
    int64_t regions;             /* distinct region numbers (or blocks of region_size vertices) */
    int64_t boundary_size;       /* |B|: vertices with a pair into another region; d_inf = max(|B|, 1) */
    int64_t boundary_pairs;      /* pairs between two regions */
    int64_t page_words;          /* int32 words per page slot (the largest region's page) */
    int64_t device_pages;        /* page slots in device memory */
    int32_t resident;            /* 1: every page lives in device memory */
    int32_t max_region_vertices;
} mf_graph_info;

typedef struct {
    int64_t max_sweeps;          /* guard; 0 = 2|B|^2 + 1 (the bound of Sec. 4.3-4.4), at least
                                  * 2^20 with round_cap > 0, where that bound does not hold */
    int32_t gap;                 /* global gap heuristic: 1 = on (the default with opts NULL), 0 = off */
    int32_t check_every;         /* resident pages: sweeps enqueued between termination checks; 0 = 8 */
    int32_t profile;             /* 1 = time every discharge launch with HIP events */
    int32_t round_cap;           /* n > 0: a region discharge runs at most n push rounds in a
                                  * sweep; its last, complete search then writes the region
                                  * relabel (Alg. 3) on the current state and a region still
                                  * holding excess that reaches a target stays active for the
                                  * next sweep; 0 = no cap (Proc. ARD to the end).  < 0: MF_E_INVAL */
} mf_graph_opts;

typedef struct {
    int64_t sweeps;              /* sweeps of Alg. 2 since the handle was created */
    int64_t discharges, push_rounds, search_steps;  /* this call's region discharges and their work */
    int64_t pages_in, pages_out; /* streamed pages: page loads and state write-backs of this call */
    int64_t bytes_h2d, bytes_d2h;
    double ms;                   /* device time of this call's sweeps (HIP events) */
    int64_t discharged_vertices, discharged_arcs;  /* summed over this call's region discharges */
    int64_t discharge_launches;  /* with opts->profile: discharge kernel launches and their */
    double discharge_ms;         /* summed duration (HIP events on the solve stream) */
} mf_graph_stats;

/* Algorithmic bytes of one region discharge of a page with nv vertices and na
 * arcs: its row offsets, heads and reverse indices read; residuals, excesses
 * and residual t-links read and written; labels written. */
int64_t mf_graph_discharge_bytes(int64_t nv, int64_t na);

/* Build a handle for the network with n vertices and npairs pairs (host
 * arrays, read during the call only): pair i joins pu[i] != pv[i] (both in
 * [0, n)) with c(pu, pv) = cuv[i] and c(pv, pu) = cvu[i]; cs[v] = c(s, v) and
 * ct[v] = c(v, t); all int32 >= 0; several pairs may join the same vertices.
 * region[v] >= 0 is the region of v (any assignment; the numbers need not be
 * dense), or region == NULL for regions of region_size consecutive vertex
 * numbers.  device_pages: 0 (or at
 * least the number of regions) keeps every page in device memory; 1 or more
 * streams the pages through that many device page slots.  The initial preflow
 * (Sec. 2: every s-link saturated, labels 0) is written into the pages.
 * Errors: MF_E_INVAL (a vertex out of range, a pair joining a vertex to
 * itself, a negative capacity or region, a page beyond 32-bit offsets, more
 * than 2^30 pairs), MF_E_OVERFLOW (c(u, v) + c(v, u), or c(s, v) plus the
 * capacities into v, above 2^31 - 1), MF_E_NOMEM, MF_E_DEVICE.  Validation
 * comes before any device call. */
mf_status mf_create_graph(int32_t n, int64_t npairs, const int32_t *pu, const int32_t *pv,
                          const int32_t *cuv, const int32_t *cvu, const int32_t *cs, const int32_t *ct,
                          const int32_t *region, int32_t region_size, int64_t device_pages,
                          mf_graph **out);
mf_status mf_graph_get_info(const mf_graph *g, mf_graph_info *info);
/* Sweeps of Alg. 2 until no vertex is active (Sec. 4.4); the preflow is then
 * maximum.  Synchronous.  opts may be NULL.  Errors: MF_E_SWEEPS (the guard
 * was reached; the state stays and a later call continues), MF_E_DEVICE. */
mf_status mf_graph_solve(mf_graph *g, const mf_graph_opts *opts, mf_graph_stats *stats);
/* |f| = sum_v f(v, t) after a completed solve, else MF_E_STATE. */
mf_status mf_graph_flow_value(const mf_graph *g, int64_t *out);
/* One byte per vertex (host array of n) in the caller's numbering: 1 on the
 * source side of the cut `kind` (MF_CUT_*), after a completed solve. */
mf_status mf_graph_min_cut(mf_graph *g, int32_t kind, uint8_t *out_source_side);
/* The state in the caller's numbering (host arrays, each may be NULL):
 * residuals of both arcs of every pair, residual t-links, excesses and
 * labels (int32 in [0, d_inf]). */
mf_status mf_graph_state(mf_graph *g, int64_t *r_uv, int64_t *r_vu, int64_t *rt, int64_t *ex,
                         int32_t *labels);
void mf_graph_destroy(mf_graph *g);

/* A DIMACS max-flow file ("p max n m", "n id s", "n id t", "a u v cap", "c"
 * comments; the problem files of the paper's experiments, Sec. 7.2) as the arrays of
 * mf_create_graph, owned by the library (mf_free_dimacs releases them).  The
 * vertices other than s and t become 0 .. n-1 in increasing file id
 * (vertex_id[i] is the file id of vertex i); an arc s -> v adds to c(s, v), an
 * arc v -> t to c(v, t), an arc s -> t to st_capacity (flow that every maximum
 * flow carries: add it to mf_graph_flow_value); every other arc u -> v becomes
 * a pair with c(u, v) = cap and c(v, u) = 0; arcs into s, out of t and from a
 * vertex to itself carry no s-t flow and are dropped.  Host code only.
 * Errors: MF_E_INVAL (unreadable file, a malformed line, an id out of range,
 * no or equal s and t, an arc count other than the problem line's),
 * MF_E_OVERFLOW (a capacity, or a vertex's summed s- or t-link, above
 * 2^31 - 1), MF_E_NOMEM. */
typedef struct {
    int32_t n;
    int64_t npairs;
    int32_t *pu, *pv, *cuv, *cvu, *cs, *ct;
    int64_t st_capacity;
    int64_t *vertex_id;
} mf_dimacs;
mf_status mf_read_dimacs(const char *path, mf_dimacs **out);
void mf_free_dimacs(mf_dimacs *d);

void mf_destroy(mf_grid *g);
const char *mf_status_str(mf_status s);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
