/*
 * gcb.h -- C ABI of the MI355X (gfx950) library for grouping-circular-based
 * (GCB) greedy RBF mesh deformation (Fang, Zhang, Shan, Tie, Zhang, Sun,
 * arXiv:2004.04817).
 *
 * The calls follow the paper's statement of the problem: Algorithm 1 takes
 * the boundary nodes G with displacements dX, dY, dZ, the group count m, the
 * allowable error E* and the support cap Nc^max, and returns the support set
 * S with weights W^x, W^y, W^z; Eq. (6) then moves any set of volume points.
 *
 * Conventions for every call:
 *  - Every function returns an int status (enum gcb_status) unless noted.
 *  - Coordinates and displacements are row-major (x, y, z) triples, float64
 *    unless a dtype argument says otherwise.
 *  - `mem` says where a pointer lives: GCB_MEM_HOST (pageable or pinned host
 *    memory) or GCB_MEM_DEVICE (device memory of the context's device).
 *  - Inputs are copied; the caller keeps ownership of every buffer it passes.
 *    Outputs go into caller-allocated buffers of the stated size.
 *  - A context is not thread-safe; use one context per thread or stream.
 *  - Device work is enqueued on the context's stream.  Calls with host
 *    outputs synchronise that stream before returning; calls with device
 *    outputs return once the work is enqueued.
 *  - On error nothing is returned through output pointers, and
 *    gcb_last_error() describes the failure.  No C++ exception crosses this
 *    interface.  GCB_E_DEVICE means a HIP runtime call failed.
 */
#ifndef GCB_H
#define GCB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gcb_ctx gcb_ctx;

enum gcb_status {
    GCB_OK = 0,
    GCB_NOT_CONVERGED = 1, /* warning: |S| reached nc_max while the error exceeded E* */
    GCB_E_INVALID = -1,    /* argument out of range, NULL pointer, non-finite input */
    GCB_E_STATE = -2,      /* call out of order (e.g. deform before select) */
    GCB_E_NOMEM = -3,      /* device or host allocation failed */
    GCB_E_SINGULAR = -4,   /* the support matrix stopped being numerically SPD */
    GCB_E_DEVICE = -5      /* a HIP runtime call failed */
};

enum gcb_mem { GCB_MEM_HOST = 0, GCB_MEM_DEVICE = 1 };
enum gcb_dtype { GCB_F32 = 0, GCB_F64 = 1 };

/* Evaluation precision of the interpolant (Eq. 1 / Eq. 6).  The support-
 * system factor, the greedy's group sweeps and decisions, and the all-node
 * certificate are FP64 in both. */
enum gcb_precision {
    GCB_PREC_FP64 = 0,       /* every evaluation in FP64 */
    GCB_PREC_FP32_EVAL = 1   /* gcb_deform evaluates Eq. (6) in FP32 (scaled coordinates, weights and
                              * phi in FP32; chunks of 32 supports summed in FP32, chunk sums in FP64).
                              * gcb_deform_batch and gcb_deform_multi stay FP64 */
};

typedef struct {
    double radius;       /* R, the Wendland C2 support radius (Eq. 2: eta = |r - r_i| / R); > 0 */
    int32_t m;           /* group count of the stochastic partition, 1 <= m <= nb (m = 1: traditional greedy) */
    uint64_t seed;       /* partition seed (splitmix64-driven Fisher-Yates shuffle) */
    double tol_abs;      /* E*, absolute allowable interpolation error (Algorithm 1); >= 0 */
    int64_t nc_max;      /* Nc^max, cap on |S|; 3 <= nc_max <= nb */
    int32_t precision;   /* enum gcb_precision */
    int32_t use_init;    /* 1: start from init_idx; 0: farthest-point rule */
    int64_t init_idx[3]; /* three distinct boundary indices when use_init = 1 */
    int32_t warm_start;  /* 1: start from the support set of the context's last finished selection
                          * (an extension of Algorithm 1 for a mesh whose boundary stays while its
                          * displacements change, see gcb_select); 0: from three starting nodes */
    int32_t monitor_every; /* > 0: after every that many loop iterations record the all-node max and RMS
                            * error with the current W (gcb_get_monitor); never alters the selection,
                            * and turns off captured chunks; not with batches.  0: off */
    int32_t per_iter;    /* nodes one iteration may append.  0 or 1: Algorithm 1.  2 ..
                          * GCB_MAX_PER_ITER: the several-nodes-per-iteration variant, a block form
                          * of the peak-selection idea cited in Section 1 (not Algorithm 1): the
                          * nodes of G_i \ S whose error exceeds E* are ranked by (error
                          * descending, original index ascending) on one sweep, and the first
                          * per_iter of them (fewer at nc_max) are appended together; an iteration
                          * with no such node is quiet, and the stopping rule is unchanged.  The
                          * log's appended[] then holds the count.  Not with warm starts, batches
                          * or the server (GCB_E_INVALID) */
    int32_t cull_volume; /* 1: gcb_deform's FP64 evaluation of Eq. (6) skips the (point, support)
                          * pairs farther apart than R, whose phi is exactly zero (Eq. 2): the
                          * points are evaluated in Morton order (a device radix sort), the
                          * supports in Morton order in tiles of 32, and a wave of 64 points skips
                          * every tile whose bounding box lies farther than R from theirs.  The
                          * sum runs over the same non-zero terms in another order (the result
                          * differs by rounding).  Device memory: 16 bytes per point.  0: off */
} gcb_params;

/* Largest per_iter of the several-nodes-per-iteration variant. */
#define GCB_MAX_PER_ITER 16

typedef struct {
    int64_t nc;              /* |S| */
    int64_t iterations;      /* greedy iterations k = 3, 4, ... that ran */
    int32_t status;          /* GCB_OK or GCB_NOT_CONVERGED */
    int32_t converged;       /* FP64 all-node max error <= E* */
    double final_max_err;    /* FP64 certificate: max_j |F(r_j) - d_j|_2 over all nb nodes */
    double final_rms_err;    /* sqrt(mean_j |F(r_j) - d_j|_2^2) */
    uint64_t pairs_group;    /* pair evaluations in the group sweeps: sum_k |G_i \ S_k| |S_k| */
    uint64_t pairs_append;   /* pair evaluations of the appended phi vectors: sum |S| */
    uint64_t pairs_cert;     /* nb * nc */
    double ms_select;        /* device wall time of the selection (hipEvents), ms */
    int64_t probed_iterations; /* of `iterations`, the trailing quiet ones that the convergence probe
                                * completed: after a run of quiet iterations (W unchanged), one FP64
                                * sweep of every group showed that each remaining iteration of
                                * Algorithm 1 appends nothing; their log entries are that sweep's
                                * group maxima.  0 when the loop ran to its end */
} gcb_select_info;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * enqueue on (NULL: the library creates its own non-blocking stream).
 * *out receives the context; release it with gcb_destroy. */
int gcb_create(gcb_ctx **out, int device, void *hip_stream);

/* Free every device and host buffer the context owns.  NULL-safe. */
void gcb_destroy(gcb_ctx *ctx);

/* Message of the last failed call on ctx (owned by ctx, valid until the next
 * call).  With ctx = NULL: the message of the last failed gcb_create. */
const char *gcb_last_error(const gcb_ctx *ctx);

/* Switch the stream later calls enqueue on: a hipStream_t, used verbatim
 * (NULL is the device's null stream, which is PyTorch's default stream).
 * Work already enqueued on the previous stream is waited for first. */
int gcb_set_stream(gcb_ctx *ctx, void *hip_stream);

/* Boundary nodes G and their prescribed displacements (Algorithm 1 input;
 * Eq. 3).  xyz and disp are (nb, 3) float64.  nb >= 3; all values finite
 * (checked).  Resets any previous selection. */
int gcb_set_boundary(gcb_ctx *ctx, int64_t nb, const double *xyz, const double *disp, int mem);

/* Replace the displacements of the same nodes, (nb, 3) float64.  The
 * previous selection's results (its weights, gcb_deform, gcb_get_support)
 * are unavailable until the next gcb_select.  Its support set S0 and the
 * factor of S0 stay in the context: a gcb_select with params.warm_start = 1
 * starts from them, one with warm_start = 0 starts afresh. */
int gcb_set_displacement(gcb_ctx *ctx, const double *disp, int mem);

/* Algorithm 1 parameters plus R (Eq. 2).  Checked against the boundary when
 * gcb_select runs. */
int gcb_set_params(gcb_ctx *ctx, const gcb_params *p);

/* Optional explicit partition: group_of[nb] in [0, m) for the current m.
 * Pass NULL to return to the seeded partition. */
int gcb_set_groups(gcb_ctx *ctx, const int32_t *group_of, int mem);

/* Run the GCB greedy selection (Algorithm 1; m = 1 is the traditional
 * greedy of Rendall and Allen).  Iteration k evaluates the interpolation
 * error of group G_{k mod m} only, and appends its maximum-error node (ties
 * to the lowest index, nodes already in S excluded) when that error exceeds
 * E* and |S| < nc_max.  It stops after m consecutive iterations without an
 * append, or when an append is refused at the cap (GCB_NOT_CONVERGED).  The
 * support system Phi_S W = Delta_S (Eqs. 4-5 restricted to S) is kept
 * factored in FP64 and extended by one row per appended node (the recurrence
 * idea of Section 1), here as the inverse factor M = L^-1.  A final FP64
 * sweep over all nb nodes fills final_max_err / final_rms_err.  info may be
 * NULL.  Returns GCB_OK, GCB_NOT_CONVERGED or an error.
 *
 * Warm start (params.warm_start = 1): the support set S0 and its factor
 * from the last finished selection stay (gcb_set_displacement keeps them;
 * gcb_set_boundary and gcb_set_groups drop them, and radius, m, seed must be
 * unchanged, else GCB_E_STATE).  The weights are recomputed for the current
 * displacements as W = M^T (M Delta_S0); if the FP64 all-node error is then
 * <= E* the selection ends with no iteration, otherwise the loop above runs
 * from k = |S0|.  nc_max must be >= |S0|. */
int gcb_select(gcb_ctx *ctx, gcb_select_info *info);

/* Selected support nodes in selection order (original boundary indices,
 * idx[nc] int64) and their weights (w[nc][3] float64); either may be NULL. */
int gcb_get_support(gcb_ctx *ctx, int64_t *idx, double *w, int mem);

/* Per-iteration record of the last selection into host arrays of length
 * cap (any may be NULL): group i = k mod m, argmax node (original index, -1
 * if the group had no candidate), its error E, appended flag.  Returns the
 * number of iterations (may exceed cap: only cap entries are written), or a
 * negative status. */
int64_t gcb_get_log(gcb_ctx *ctx, int32_t *group, int64_t *node, double *err, int8_t *appended, int64_t cap);

/* Eq. (6): displacements of nv arbitrary points from the selected supports:
 * out[k] = sum_{s in S} w_s phi(|r_k - r_s| / R).  xyz (nv, 3) of in_dtype,
 * out (nv, 3) of out_dtype (GCB_F32 or GCB_F64), both in `mem`.  Arithmetic
 * is FP64 (unless GCB_PREC_FP32_EVAL): squared distances from coordinates
 * centred at the first support, the square root to about 1e-14 relative, so
 * each phi is within about 1e-13 of its exact value.  The first FP64 call
 * allocates a device table of 32 bytes per support capacity, kept by the
 * context.  nv = 0 is a no-op.  Requires a finished gcb_select. */
int gcb_deform(gcb_ctx *ctx, int64_t nv, const void *xyz, int in_dtype, void *out, int out_dtype, int mem);

/* Measurement aid for the greedy loop's kernels (Algorithm 1's group sweep,
 * and the two kernels of the support-system append of Section 1's RC
 * scheme: the decision with l = M b, and u = M^T l with the new factor row).
 * With on = 1, later gcb_select calls run their iterations without captured
 * graphs and record HIP events on the context's stream between the launches
 * of every iteration's kernels, and around the all-node certificate; the
 * selection is slower, its results are the same.  on = 0 turns it off. */
int gcb_set_kernel_timing(gcb_ctx *ctx, int32_t on);

/* Device time of the last selection that ran with kernel timing on:
 * ms[0..3] summed milliseconds and launches[0..3] launch counts of the group
 * sweep (k_sweep, k_sweep_wide or k_sweep_lanes), k_factor_l, k_factor_u and
 * the all-node certificate (k_certify with its final reduction); either
 * pointer may be NULL.  An interval runs from the event before a launch to
 * the event after it, so it includes that launch's dispatch on the device.
 * GCB_E_STATE if no selection ran with kernel timing on. */
int gcb_get_kernel_times(gcb_ctx *ctx, double *ms, int64_t *launches);

/* Pairs of the last culled deformation (params.cull_volume = 1): *evaluated
 * (point, support) pairs the sweep computed, *dense = nv x nc (the pairs the
 * plain sweep computes); either may be NULL.  Waits for the deformation.
 * GCB_E_STATE if no culled deformation has run. */
int gcb_get_deform_pairs(gcb_ctx *ctx, uint64_t *evaluated, uint64_t *dense);

/* Largest support count gcb_deform_noalloc accepts. */
#define GCB_NOALLOC_MAX_SUPPORTS 8192

/* Allocation-free form of gcb_deform, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops or harnesses
 * that forbid hipMalloc).  Same result as gcb_deform with mem =
 * GCB_MEM_DEVICE, bitwise: the same kernels, in the context's precision.
 * xyz (nv, 3) of in_dtype and out (nv, 3) of out_dtype are device memory on
 * the context's device, owned by the caller.  The per-call support table
 * (FP64: 32 bytes per support; FP32 evaluation: 24 bytes) is kept in one
 * static device array of GCB_NOALLOC_MAX_SUPPORTS entries per GPU (256 KiB,
 * held until the process ends) instead of context buffers: the call makes
 * no device allocation, copy or event.  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (other contexts, other streams)
 * race.  Returns GCB_E_INVALID when the selection has more than
 * GCB_NOALLOC_MAX_SUPPORTS supports (gcb_deform has no such limit),
 * GCB_E_STATE without a finished selection.  gcb_deform_time does not time
 * it.  nv = 0 is a no-op. */
int gcb_deform_noalloc(gcb_ctx *ctx, int64_t nv, const void *xyz, int in_dtype, void *out, int out_dtype);

/* Device time (*ms, milliseconds) of the kernels of the last gcb_deform,
 * between two events on the context's stream (host copies excluded; not
 * recorded while the stream is being captured).  Waits for the second event.
 * GCB_E_STATE if no timed deformation has run. */
int gcb_deform_time(gcb_ctx *ctx, double *ms);

/* Multiple right-hand sides on one support set: k_modes displacement fields
 * of the same boundary nodes, disp_modes (nb, 3*k_modes) float64 (columns
 * x, y, z of mode 0, then mode 1, ...), are solved on the selected S (Eqs.
 * 4-5 restricted to S, FP64 factor) and evaluated at nv points (Eq. 6):
 * out (nv, 3*k_modes) of out_dtype.  Requires a finished gcb_select. */
int gcb_deform_multi(gcb_ctx *ctx, int32_t k_modes, const double *disp_modes, int64_t nv, const void *xyz,
                     int in_dtype, void *out, int out_dtype, int mem);

/* Give the context a support set instead of selecting one: idx[0..n) are
 * distinct boundary indices (host or device memory per mem), 3 <= n <=
 * nc_max.  The support system Phi_S (Eqs. 4-5 restricted to S, in this
 * order) is factored from scratch in FP64 (Cholesky factor and its inverse
 * M = L^-1 by recursive halving, the block products on the matrix cores;
 * Section 2: Phi is SPD), W = M^T (M Delta_S) for the current
 * displacements, and the FP64 all-node certificate fills *info (may be
 * NULL; iterations = 0).  Afterwards the context is as after a finished
 * selection: gcb_deform, gcb_get_support and warm starts work.  Returns
 * GCB_OK, GCB_E_SINGULAR (a pivot <= 64 DBL_EPSILON) or an error. */
int gcb_set_support(gcb_ctx *ctx, const int64_t *idx, int64_t n, int mem, gcb_select_info *info);

/* Monitor samples of the last selection (params.monitor_every = E > 0):
 * sample s was taken after loop iteration (s + 1) E (counted from the loop
 * start), with the weights of that moment: iteration[s] = (s + 1) E,
 * max_err[s] / rms_err[s] = max / RMS over all nb nodes of |F(r_j) - d_j|_2
 * (Section 3: after m iterations every node has been checked once).  Any
 * array may be NULL; up to cap samples are written.  Returns the number of
 * samples, or a negative status. */
int64_t gcb_get_monitor(gcb_ctx *ctx, int64_t *iteration, double *max_err, double *rms_err, int64_t cap);

/* Copy out the inverse factor M = L^-1 of the current support set (Phi_S =
 * L L^T in selection order) as packed rows: row i, entries 0..i, starts at
 * i(i+1)/2; m holds nc(nc+1)/2 doubles (host or device per mem). */
int gcb_get_factor(gcb_ctx *ctx, double *m, int mem);

/* Re-certify the inverse factor of the current support set against rounding
 * drift: rebuild it from scratch as in gcb_set_support, replace the grown
 * one, recompute W and the certificate (in *info, may be NULL).  *drift (may
 * be NULL) gets max|M_new - M_old| / max|M_old| over the packed factor. */
int gcb_refactor(gcb_ctx *ctx, double *drift, gcb_select_info *info);

/* FP64 interpolation error over all nb boundary nodes with the current
 * support set (the convergence certificate): max and RMS of |F(r_j) - d_j|_2. */
int gcb_certify(gcb_ctx *ctx, double *max_err, double *rms_err);

/* ------------------------------------------------------------------
 * Batches: several independent surfaces advanced by shared launches.
 * One greedy iteration of every running context of a batch is three kernel
 * launches in total, whatever the number of contexts, so the launch latency
 * that bounds a single selection is shared (uneven surfaces, continuous
 * batching of requests).  Each context keeps its own state, support set and
 * factor; results equal those of gcb_select on the same context.
 * ------------------------------------------------------------------ */
typedef struct gcb_batch gcb_batch;

/* Create a batch on HIP device `device` that enqueues on the hipStream_t
 * `hip_stream`, taken verbatim (NULL is the null stream).  Release with
 * gcb_batch_destroy. */
int gcb_batch_create(gcb_batch **out, int device, void *hip_stream);
void gcb_batch_destroy(gcb_batch *b);   /* NULL-safe; contexts are not touched */
const char *gcb_batch_last_error(const gcb_batch *b);

/* Launch layout (tile shapes) of the batched iterations, chosen by an
 * autotuner or left automatic.  sweep_tpl: targets per lane in the group
 * sweeps (1, 2 or 4 with one wave per target group; 0: automatic);
 * factor_rpw: 16-row chunks of M per factor wave (1 or 4; 0: automatic);
 * lone_graph: 1 (default) lets a step with a single running context replay
 * that context's captured chunk of iterations.  factor_rpw changes no result;
 * sweep_tpl changes only the summation order of the group errors. */
int gcb_batch_set_layout(gcb_batch *b, int32_t sweep_tpl, int32_t factor_rpw, int32_t lone_graph);

/* Start the selection of ctx (boundary and parameters set, same device as
 * the batch): partition and staging, the three starting nodes.  ctx is
 * switched to the batch's stream.  Errors are those of gcb_select; the
 * message is in gcb_last_error(ctx). */
int gcb_batch_begin(gcb_batch *b, gcb_ctx *ctx);

/* Run `iterations` (1..4096) further greedy iterations of every listed
 * context whose selection is in progress (at most 64 of them), in shared
 * launches; the host waits for the batch's stream first.  running[i]
 * (may be NULL) gets 1 while context i still runs.  Returns the number of
 * contexts still running, or a negative status (message in the failing
 * context's gcb_last_error, or in gcb_batch_last_error). */
int32_t gcb_batch_step(gcb_batch *b, gcb_ctx *const *ctxs, int32_t count, int32_t iterations, int32_t *running);

/* Finish a context whose selection stopped: FP64 certificate over all its
 * boundary nodes, result in *info (may be NULL).  Returns GCB_OK,
 * GCB_NOT_CONVERGED or an error (GCB_E_STATE if it is still running). */
int gcb_batch_end(gcb_batch *b, gcb_ctx *ctx, gcb_select_info *info);

/* begin + step until none runs + end, for `count` contexts, in slices of at
 * most 64 contexts; infos[i] (array may be NULL) gets each result.  Returns
 * GCB_OK, GCB_NOT_CONVERGED if any context hit its cap, or the first error. */
int gcb_select_batch(gcb_batch *b, gcb_ctx *const *ctxs, int32_t count, gcb_select_info *infos);

/* Eq. (6) for every context in one launch: context i moves nv[i] points
 * xyz[i] (nv[i] x 3 of in_dtype) into out[i] (nv[i] x 3 of out_dtype).  All
 * pointers are device memory of the batch's device; every context needs a
 * finished selection. */
int gcb_deform_batch(gcb_batch *b, gcb_ctx *const *ctxs, int32_t count, const int64_t *nv, const void *const *xyz,
                     int in_dtype, void *const *out, int out_dtype);

/* ------------------------------------------------------------------
 * Serving: a request loop over deformation requests of different sizes.
 * Requests wait in FIFO order and are admitted as slots (max_active) and the
 * device-memory budget allow.  With GCB_SERVE_BATCH the admitted selections
 * advance together in shared launches (gcb_batch_step), new requests joining
 * at the next step (continuous batching), and finished ones are deformed in
 * one batched volume launch; without it, each admitted request runs
 * gcb_select and gcb_deform on its own, one at a time.  With GCB_SERVE_CACHE
 * a finished mesh (keyed by mesh_key) stays resident with its support set
 * and factor; a later request with the same key, the same boundary and new
 * displacements is served by a warm start (see gcb_select).  Idle resident
 * meshes are evicted, least recently used first, when a new mesh would
 * exceed the budget.  Every result equals that of the same call sequence on
 * a context of its own.
 * ------------------------------------------------------------------ */
typedef struct gcb_server gcb_server;

enum gcb_serve_flags { GCB_SERVE_BATCH = 1, GCB_SERVE_CACHE = 2 };

/* What a request's selection produced, copied into caller-owned host
 * arrays when the selection finishes (Algorithm 1's outputs S and W plus its
 * per-iteration record, as gcb_get_support and gcb_get_log give them for a
 * context of its own).  The copies synchronise the server's stream, so a
 * recorded request delays the rounds that finish it: meant for verification,
 * not for timed streams.  Arrays may be NULL; at most cap_support supports
 * and cap_log iterations are written; nc and iterations are filled in. */
typedef struct {
    int64_t cap_support;     /* entries support[] (and rows of weights[]) can hold */
    int64_t *support;        /* selected nodes, original boundary indices, selection order */
    double *weights;         /* (cap_support, 3): W^x, W^y, W^z */
    int64_t cap_log;         /* entries each log array can hold */
    int32_t *log_group;      /* group k mod m of each iteration of this request's loop */
    int64_t *log_node;       /* its argmax node (original index, -1: no candidate) */
    double *log_err;         /* the group maximum error E */
    int8_t *log_appended;    /* 1: the node was appended */
    int64_t nc;              /* out: |S| */
    int64_t iterations;      /* out: loop iterations of this request (0 for a warm start that met E*) */
} gcb_record;

typedef struct {
    int64_t mesh_key;        /* >= 0: identity of the boundary for the resident cache; -1: never kept */
    int64_t nb;              /* boundary nodes */
    const double *xyz;       /* (nb, 3) host memory, read at admission */
    const double *disp;      /* (nb, 3) host memory, read at admission */
    gcb_params params;       /* as for gcb_set_params; the server sets warm_start itself */
    int64_t nv;              /* volume points (0: selection only) */
    const void *vol_xyz;     /* (nv, 3) of in_dtype, device memory */
    int32_t in_dtype;        /* GCB_F32 or GCB_F64 */
    int32_t out_dtype;       /* GCB_F32 or GCB_F64 */
    void *out;               /* (nv, 3) of out_dtype, device memory: the displacements of Eq. (6) */
    double t_arrival;        /* arrival time on gcb_server_clock(); < 0: the time of submission */
    gcb_record *record;      /* NULL, or host memory filled when the selection finishes (valid until done) */
} gcb_request;

typedef struct {
    int32_t state;           /* 0 queued, 1 selecting, 2 deforming, 3 done; < 0: failed with this status */
    int32_t warm;            /* 1: served by a warm start from a resident support set */
    int32_t kept;            /* 1: its mesh stays resident afterwards (until evicted) */
    int32_t reserved;
    gcb_select_info info;    /* the selection's result (state 3) */
    double t_arrival;        /* server clock, seconds */
    double t_admit;          /* admission (slot and memory granted) */
    double t_done;           /* the output is complete on the device (event time mapped to the clock) */
} gcb_result;

/* Monotonic clock of the server, seconds. */
double gcb_server_clock(void);

/* Create a server on `device` enqueueing on `hip_stream` (verbatim; NULL is
 * the null stream).  hbm_budget: device bytes the resident and running
 * meshes may hold (a soft cap: a request is admitted alone when nothing else
 * runs); max_active: 1..64 concurrent selections; flags: gcb_serve_flags. */
int gcb_server_create(gcb_server **out, int device, void *hip_stream, uint64_t hbm_budget, int32_t max_active,
                      int32_t flags);
void gcb_server_destroy(gcb_server *s);   /* NULL-safe; waits for the device */
const char *gcb_server_last_error(const gcb_server *s);

/* Queue a request (arguments are checked now; buffers must stay valid
 * until its result reaches state 3 or fails).  *ticket identifies it. */
int gcb_server_submit(gcb_server *s, const gcb_request *req, int64_t *ticket);

/* One scheduling round: record finished outputs, admit waiting requests,
 * run `iterations` (1..4096) greedy iterations of every admitted selection,
 * finish and deform those that stopped.  *in_flight (may be NULL) gets the
 * number of requests not yet done.  A failing request is marked failed;
 * the round goes on. */
int gcb_server_progress(gcb_server *s, int32_t iterations, int32_t *in_flight);

/* The state and timings of a ticket. */
int gcb_server_result(const gcb_server *s, int64_t ticket, gcb_result *res);

/* Drop the record of a finished (state 3) or failed ticket, so that a server
 * that runs for long keeps a bounded amount of host memory; the ticket is
 * unknown afterwards (GCB_E_INVALID).  GCB_E_STATE while it is still queued
 * or running. */
int gcb_server_forget(gcb_server *s, int64_t ticket);

/* Device bytes held by resident and running meshes, and the resident count. */
int gcb_server_memory(const gcb_server *s, uint64_t *bytes, int32_t *resident);

/* Host-only: the seeded partition the library uses (Section 3: groups
 * pairwise disjoint, sizes differ by at most one).  Fisher-Yates shuffle pi
 * of 0..nb-1 driven by splitmix64(seed), node pi[t] to group t mod m.
 * group_of[nb] host int32.  Makes no HIP call. */
int gcb_partition(int64_t nb, int32_t m, uint64_t seed, int32_t *group_of);

/* Host-only: library version string (static storage). */
const char *gcb_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GCB_H */
