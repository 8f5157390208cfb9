/*
 * qtn.h — C ABI of the MI355X bucket-elimination library for the QAOA MaxCut
 * energy expectation (arXiv 2204.06045, "Performance Evaluation and
 * Acceleration of the QTensor Quantum Circuit Simulator on GPUs").
 *
 * What it computes (Sec. II-A, Eq. 1 and Eq. 2; Sec. II-B):
 *   |gamma,beta>_p = prod_{l=1..p} exp(-i beta_l B) exp(-i gamma_l C) |+>^N,
 *   C = 1/2 sum_{(jk) in E} (1 - Z_j Z_k),  B = sum_i X_i,
 *   e_jk = <gamma,beta| Z_j Z_k |gamma,beta>,
 *   E    = <C> = |E|/2 - 1/2 sum_jk e_jk.
 * Each e_jk is the scalar of one light-cone tensor network (Sec. II-B),
 * contracted by bucket elimination (Sec. II-B): buckets are taken in the
 * elimination order, the tensors of a bucket are multiplied over the union of
 * their binary indices and the bucket index is summed out.  Consecutive
 * buckets whose index sets nest are merged and summed in one pass (merged
 * indices, Sec. II-C).
 *
 * Conventions for every call:
 *   - returns QTN_OK (0) or a negative QTN_E* code; qtn_last_error() gives a
 *     message for the calling thread, valid until its next call;
 *   - no C++ exception crosses this boundary: a failed host allocation
 *     returns QTN_ENOMEM, any other internal exception QTN_EINVAL with a
 *     message starting "internal error";
 *   - on error, caller-owned output buffers are left untouched;
 *   - arrays passed in are copied; the caller keeps ownership;
 *   - a qtn_network is owned by the library and released by
 *     qtn_network_free; calls on one network are not thread-safe.
 */
#ifndef QTN_H
#define QTN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QTN_OK 0
#define QTN_EINVAL (-1)  /* bad graph, angle, order or argument            */
#define QTN_ERANGE (-2)  /* bucket width or memory over the configured cap */
#define QTN_ENOMEM (-3)  /* workspace too small or host allocation failed  */
#define QTN_EDEVICE (-4) /* HIP runtime error (message has the HIP string) */
#define QTN_ESTATE (-5)  /* call order (e.g. contract before plan)        */

/* Arithmetic of the contraction. */
#define QTN_C128 0  /* complex128 throughout                             */
#define QTN_C64 1   /* complex64 buckets, FP64 scalars and energy        */
#define QTN_MIXED 2 /* complex64 for groups of union width >= mixed_width
                       (their outputs stored as complex64), complex128 for
                       the rest and for every group ending in a scalar;
                       operands convert on load                          */

typedef struct qtn_network qtn_network;

/* Tunables; zero fields take the defaults given in brackets. */
typedef struct qtn_config {
    int32_t max_levels;  /* bucket indices summed per fused group, 1..8 [8];
                            1 = plain per-bucket contraction (no merging)   */
    int32_t small_width; /* groups of union width <= this run inside one
                            workgroup, many per launch [12]                */
    int32_t max_width;   /* refuse plans with a bucket wider than this [32] */
    int32_t n_streams;   /* HIP streams the light cones are spread over [4] */
    int32_t eager;       /* 1: launch eagerly instead of replaying a
                            captured HIP graph [0]                          */
    int32_t lane_sum_bits; /* streaming kernel: summed indices spread over
                            lanes, the rest walked serially per lane [2];
                            with variant 4, the cell mapping's cell bits
                            (2..4, else 3)                                 */
    int32_t variant;     /* 0 auto (the cell mapping for own-launch groups
                            it fits in the per-group launch executors,
                            else streaming or generic), 1 generic kernel
                            only, 2 streaming kernel wherever it applies,
                            3 matrix form for every group that has one
                            (complex128 in own launches; complex64 also in
                            workgroups and the persistent executors;
                            others as auto), 4 cell mapping wherever it
                            applies [0]                                     */
    int32_t order_trials; /* >1: plan with the cheapest (sum of 2^width) of
                            the greedy min-fill order and order_trials-1
                            min-fill orders with random tie-breaks [0]     */
    int32_t executor;    /* 0 default (single networks: per-group launches
                            over n_streams; batches: persistent lockstep),
                            1 per-group launches, 2 one persistent lockstep
                            launch, 3 per-group launches with each cone's
                            leading small groups launched on that cone's
                            stream, 4 one persistent dataflow launch (work
                            items wait only for the previous task of their
                            own light cone), 5 hybrid: one persistent
                            lockstep launch for the light cones, then
                            per-group launches for the heavy ones
                            (hybrid_width)                                 */
    int32_t spin_limit;  /* persistent executors: polls before a barrier or
                            dependency wait gives up with QTN_EDEVICE [2^22] */
    int32_t mixed_width; /* QTN_MIXED: narrowest group run in complex64 [18] */
    int32_t slice_width; /* >0: index slicing for every light cone whose
                            widest bucket exceeds this width: up to 10 of its
                            variables are fixed (greedily, from its widest
                            bucket, until the width fits or nothing more can
                            be fixed), each value combination (a slice) is
                            contracted in turn on one arena and e_jk is the
                            FP64 sum of the slices' scalars; 0 off [0]      */
    int32_t order_weight; /* order_trials > 1: 0 picks the order with the
                            smallest sum of 2^width [0]; > 0 the one whose
                            merged plan has the smallest complex flops +
                            order_weight * algorithmic bytes (the groups the
                            kernels run, in the plan's precision)          */
    int32_t hybrid_width; /* executor 5: light cones whose widest bucket is
                            at most this run in one persistent lockstep
                            launch, the others after it by per-group
                            launches (cell mapping allowed) on the side
                            streams; their leading small groups, which
                            need no other group, run in the persistent
                            launch's first step [20]                       */
    int32_t reserved[2];
} qtn_config;

/*
 * Build the per-edge light-cone networks (Sec. II-B) of graph G for depth p.
 *   n_vertices  N >= 2
 *   n_edges     |E| >= 1
 *   edges       [n_edges][2] vertex ids, 0 <= u,v < N, u != v, no repeats
 *   gamma,beta  [p] angles in radians, finite (Eq. 2)
 *   cfg         NULL for defaults
 *   out         receives the network handle
 * The light cone of edge (j,k) keeps, at layer l, the mixers on vertices
 * within graph distance p-l of {j,k} and the cost gates on edges with an
 * endpoint there; every other gate cancels against its conjugate.
 * Errors: QTN_EINVAL for a bad graph or angle; QTN_ENOMEM.
 */
int qtn_network_build(int32_t n_vertices, int64_t n_edges, const int32_t *edges,
                      int32_t p, const double *gamma, const double *beta,
                      const qtn_config *cfg, qtn_network **out);

/* Size of the light cone of one edge: variables, tensors and the width of the
 * widest bucket under the greedy min-fill order. */
int qtn_network_info(const qtn_network *net, int64_t edge, int32_t *n_vars,
                     int32_t *n_tensors, int32_t *width_minfill);

/*
 * Greedy min-fill elimination order of one light cone (Sec. II-B orders the
 * buckets; the paper leaves the heuristic open).  Ties go to the fewest
 * remaining neighbours, then the smallest variable id; variables are numbered
 * in creation order: starting variables by vertex, then per layer the new
 * ket variables by vertex, then the bra variables from layer p down to 1.
 *   order_out  [n_vars] receives a permutation of 0..n_vars-1
 */
int qtn_order_minfill(const qtn_network *net, int64_t edge, int32_t *order_out);

/*
 * Plan the contraction: symbolic bucket elimination, merged-index groups
 * (Sec. II-C), memory plan and kernel schedule.
 *   orders     NULL (min-fill for every edge) or [n_edges] pointers, each NULL
 *              (min-fill) or a permutation of that light cone's variables
 *   precision  QTN_C128, QTN_C64 or QTN_MIXED
 *   workspace_bytes_out  device bytes qtn_contract needs
 * Errors: QTN_EINVAL (order not a permutation), QTN_ERANGE (width over cap).
 */
int qtn_plan(qtn_network *net, const int32_t *const *orders, int32_t precision,
             size_t *workspace_bytes_out);

/* The elimination order qtn_plan used for one light cone. */
int qtn_plan_order(const qtn_network *net, int64_t edge, int32_t *order_out);

/* Replace the angles (values only; the plan is kept). */
int qtn_set_angles(qtn_network *net, const double *gamma, const double *beta);

/*
 * Contract every light cone on the GPU.
 *   d_workspace  device memory of at least the planned size, owned by the
 *                caller, 256-byte aligned, live until this call returns
 *   hip_stream   hipStream_t to order the work after (NULL = null stream)
 *   zz_out       [n_edges] Re e_jk
 *   zz_imag_out  [n_edges] Im e_jk (zero up to rounding) or NULL
 *   energy_out   <C> = |E|/2 - 1/2 sum Re e_jk, accumulated in FP64
 * Blocks until the results are on the host.
 * Errors: QTN_ESTATE (no plan), QTN_ENOMEM (workspace too small),
 *         QTN_EDEVICE.
 */
int qtn_contract(qtn_network *net, void *d_workspace, size_t bytes,
                 void *hip_stream, double *zz_out, double *zz_imag_out,
                 double *energy_out);

/*
 * Contract several planned networks in one batch: all of their light cones
 * share one workspace and one launch sequence.
 *   nets         [n] planned networks of one precision
 *   d_workspace  at least qtn_batch_workspace() bytes
 *   zz_out       concatenated [sum n_edges] Re e_jk, network by network
 *   energy_out   [n]
 */
int qtn_contract_batch(qtn_network *const *nets, int32_t n, void *d_workspace,
                       size_t bytes, void *hip_stream, double *zz_out,
                       double *energy_out);

/* Workspace bytes qtn_contract_batch needs for these networks. */
int qtn_batch_workspace(qtn_network *const *nets, int32_t n,
                        size_t *workspace_bytes_out);

/* Schedule search for a batched call (the small-bucket overhead of a batch
 * of networks, Sec. III-C): the persistent lockstep launch's grid (all
 * resident blocks, three quarters or half of them, in whole rounds over the
 * 8 XCDs) and the order of the work items inside each lockstep step (the
 * costliest light cone's first, or reversed).  Each of the 6 configurations
 * runs qtn_contract_batch 4 times on d_workspace; the best of the last 3
 * host-clock call times is its time.  The configuration built first is
 * kept unless another is more than 3% faster.  The choice stays with this
 * list of networks (the schedule that later qtn_contract_batch calls on the
 * same networks, unplanned since, reuse).  Results are the same in every
 * configuration: each item computes the same values, whichever block runs it.
 *   nets, n, d_workspace, bytes, hip_stream: as for qtn_contract_batch
 *   report  filled if not NULL
 * QTN_ESTATE unless the networks use executor 0, 2 or 5 (the lockstep and
 * hybrid forms); errors of the calls as for qtn_contract_batch. */
typedef struct qtn_batch_tune_report {
    int32_t n_candidates;   /* configurations measured (6)                */
    int32_t pick;           /* the one kept                               */
    int32_t grid_blocks[8]; /* persistent grid of each                    */
    int32_t item_order[8];  /* 0 costliest cone's items first, 1 reversed */
    double ms[8];           /* best call time of each (milliseconds)      */
} qtn_batch_tune_report;

int qtn_autotune_batch(qtn_network *const *nets, int32_t n, void *d_workspace,
                       size_t bytes, void *hip_stream, qtn_batch_tune_report *report);

/* Per-kernel-class timing of one eager evaluation, for the roofline report. */
#define QTN_NKERNELS 5
#define QTN_K_FILL 0       /* gate-table fill from the angles            */
#define QTN_K_BLOCK 1      /* small groups, many per workgroup            */
#define QTN_K_WIDE 2       /* one wide group per launch                   */
#define QTN_K_REDUCE 3     /* per-edge scalars and the energy             */
#define QTN_K_PERSISTENT 4 /* every group in one lockstep launch          */
typedef struct qtn_timing {
    double ms[QTN_NKERNELS];        /* summed launch durations (HIP events) */
    int64_t launches[QTN_NKERNELS]; /* launches per class                 */
    double bytes[QTN_NKERNELS];     /* algorithmic HBM bytes per class    */
    double flops[QTN_NKERNELS];     /* complex-arithmetic FLOPs per class */
} qtn_timing;

/* Like qtn_contract, but eager, with every launch serialized on one stream
 * and bracketed by its own HIP event pair, so that each pair times one kernel
 * alone; fills *timing.  Slower than qtn_contract by the event overhead and
 * the lost overlap; the kernels and the schedule are the same. */
int qtn_contract_timed(qtn_network *net, void *d_workspace, size_t bytes,
                       void *hip_stream, double *zz_out, double *energy_out,
                       qtn_timing *timing);

/*
 * Several angle sets on one plan in one pass: every launch of the schedule
 * covers all sets, so each launch carries n_sets times the work (a parameter
 * search evaluates many (gamma, beta) on one graph, Sec. II-A).
 *   n_sets       1..1024
 *   gamma, beta  [n_sets][p] angles in radians, finite
 *   zz_out       [n_sets][n_edges] Re e_jk, or NULL
 *   energy_out   [n_sets] energies, or NULL
 * The workspace (qtn_angles_workspace) holds one copy of every intermediate
 * per set.  Runs the per-group launch schedule (executor 0, 1 or 3 behaviour)
 * on the network's streams; blocks until the results are on the host.
 * The network's own angles (qtn_set_angles) are not used or changed.
 *   timing_out   NULL, or: launches serialized on one stream and timed as in
 *                qtn_contract_timed (fills it and the launch log; bytes and
 *                flops cover all sets)
 * Errors: QTN_EINVAL (n_sets or angles), QTN_ESTATE, QTN_ENOMEM, QTN_EDEVICE.
 */
int qtn_angles_workspace(qtn_network *net, int32_t n_sets, size_t *workspace_bytes_out);
int qtn_contract_angles(qtn_network *net, void *d_workspace, size_t bytes,
                        void *hip_stream, int32_t n_sets, const double *gamma,
                        const double *beta, double *zz_out, double *energy_out,
                        qtn_timing *timing_out);

/*
 * Energy and its gradient in (gamma, beta) for a parameter search (Sec. II-A:
 * the energy is maximised over the angles): central differences
 * dE/dgamma_l = (E(gamma_l + h) - E(gamma_l - h)) / 2h, the same for beta_l,
 * with the 4p + 1 angle sets (the given angles and each shifted one) evaluated
 * in one qtn_contract_angles pass on the network's plan.  The network's own
 * angles (qtn_set_angles) are not changed.
 *   gamma, beta     [p] radians (host)
 *   step            h > 0; the truncation error is O(h^2), the rounding error
 *                   O(eps |E| / h) (about 1e-4 .. 1e-3 in complex128)
 *   energy_out      E at the given angles
 *   grad_*_out      [p] (host)
 * qtn_gradient_workspace stores the workspace bytes (that of 4p + 1 sets).
 * Errors: as qtn_contract_angles; QTN_EINVAL also for a bad step.
 */
int qtn_gradient_workspace(qtn_network *net, size_t *workspace_bytes_out);
int qtn_energy_gradient(qtn_network *net, void *d_workspace, size_t bytes,
                        void *hip_stream, const double *gamma, const double *beta,
                        double step, double *energy_out, double *grad_gamma_out,
                        double *grad_beta_out);

/* One launch of the last qtn_contract_timed call on this network. */
typedef struct qtn_launch_rec {
    int32_t kind;      /* QTN_K_* class                                   */
    int32_t group;     /* first group of the launch (plan order)          */
    int32_t n_groups;  /* groups in the launch                            */
    int32_t w, L;      /* union width and summed indices (first group)    */
    int32_t n_ops;     /* operands of the first group                     */
    int32_t variant;   /* kernel mapping of the first group: 0 generic,
                          1 streaming, 2 matrix form, 3 cells              */
    int32_t n_units;   /* wave units of the first group                   */
    int32_t prec;      /* arithmetic of the first group: QTN_C128/QTN_C64 */
    int32_t cvt;       /* 1: some operand of it is stored in the other
                          precision and converted on load                 */
    int32_t knob;      /* streaming: lane-summed bits; cells: cell bits;
                          matrix form: 16-column blocks per tile        */
    int32_t serial;    /* streaming and cells: serially walked summed bits */
    double ms;         /* HIP-event duration                              */
    double bytes;      /* algorithmic bytes of the launch                 */
    double flops;      /* complex-arithmetic FLOPs of the launch          */
} qtn_launch_rec;

/* Copies up to `cap` records of the last timed evaluation into `out` and
 * stores the number available in *n_out. */
int qtn_launch_log(const qtn_network *net, int64_t cap, qtn_launch_rec *out,
                   int64_t *n_out);

/* Kernel variants a group can run with (cost-model outputs). */
#define QTN_VAR_BLOCK 0   /* inside one workgroup, many groups per launch  */
#define QTN_VAR_STREAM 1  /* own launch, streaming family: the cell mapping
                             (lanes on the low union bits, register
                             cells, LDS offset tables, reduce-scatter) or
                             the lane-sum streaming mapping (LDS lane
                             tables, serial walk, butterflies)           */
#define QTN_VAR_GENERIC 2 /* own launch, generic register/lane mapping   */
#define QTN_VAR_MFMA 3    /* matrix form on the matrix cores (groups whose
                             operands split into two sides)               */

typedef struct qtn_tune_report {
    int32_t n_groups;     /* own-launch groups tuned                        */
    int32_t n_candidates; /* configurations measured                        */
    double cand_ms[8];    /* summed own-launch group time per configuration
                             (the matrix form: over the groups that have
                             one; 0 when none has)                          */
    double tuned_ms;      /* the same with each group's fastest choice      */
    int32_t picks[8];     /* groups that chose each configuration           */
} qtn_tune_report;

/*
 * Autotuner.  Runs the planned evaluation once per candidate configuration
 * (generic mapping; streaming mapping with 1, 2 or 3 lane-summed bits; matrix
 * form, which only the groups that have one take part in; cell mapping with
 * 3 or 4 cell bits, for the groups wide enough for it), each group in
 * its own launch on one stream and, for groups up to width 16, again alone
 * inside one workgroup, timing every launch with HIP events.  Each group then
 * keeps its fastest configuration for where it runs, and the plan's schedule
 * is rebuilt.  Needs the workspace qtn_plan reported.  The timings
 * are kept for qtn_tune_log.  Results of qtn_contract are unchanged up to
 * rounding order.
 */
int qtn_autotune(qtn_network *net, void *d_workspace, size_t bytes,
                 void *hip_stream, qtn_tune_report *report);

/*
 * The same autotuner with every candidate run over `n_sets` copies of the
 * network's current angles in one pass (the launches of qtn_contract_angles),
 * so that each group keeps the kernel that is fastest for angle batches of
 * that size; the tuned choices then serve single calls and batches alike.
 * qtn_tune_angles_workspace stores the workspace bytes it needs (the largest
 * candidate schedule at that set count).
 * Errors: QTN_EINVAL (n_sets outside 1..1024), QTN_ESTATE, QTN_ENOMEM (host
 * allocation, or a workspace smaller than needed), QTN_EDEVICE.
 */
int qtn_tune_angles_workspace(qtn_network *net, int32_t n_sets, size_t *workspace_bytes_out);
int qtn_autotune_angles(qtn_network *net, void *d_workspace, size_t bytes,
                        void *hip_stream, int32_t n_sets, qtn_tune_report *report);

/* One group's timings from the last qtn_autotune: its 16 shape features and
 * the measured time of each QTN_VAR_* (negative: not measured). */
typedef struct qtn_tune_rec {
    float features[16];
    double ms[4];
} qtn_tune_rec;

int qtn_tune_log(const qtn_network *net, int64_t cap, qtn_tune_rec *out,
                 int64_t *n_out);

/* One group's kernel choice, as set by qtn_autotune or qtn_apply_costmodel
 * (-1 fields: the width rule decides).  `shape` fingerprints the group (width,
 * summed indices and operand index sets) so that a stored choice is only ever
 * applied to the same group of the same plan. */
typedef struct qtn_tune_pick {
    int32_t edge;     /* light cone */
    int32_t group;    /* group index inside the light cone's plan */
    int8_t place;     /* 0 inside a workgroup segment, 1 own launch, -1 rule */
    int8_t variant;   /* 1 generic, 2 streaming, 3 matrix form, 4 cells,
                         -1 rule (a mapping that does not fit the group
                         falls back to the rule) */
    int8_t rls;       /* streaming: lane-summed bits; cells: cell bits;
                         -1 rule */
    int8_t pad;
    uint32_t shape;
} qtn_tune_pick;

/* Copies up to `cap` picks (one per group, all light cones in order) into
 * `out` and stores the number of groups in *n_out.  Lets a tuning result be
 * stored and reapplied to a later plan of the same network, order and
 * precision without measuring again. */
int qtn_tune_picks(const qtn_network *net, int64_t cap, qtn_tune_pick *out,
                   int64_t *n_out);

/* Applies stored picks and rebuilds the schedule.  Every pick must name an
 * existing group whose shape matches; otherwise nothing is applied and the
 * call fails with QTN_EINVAL. */
int qtn_set_tune_picks(qtn_network *net, const qtn_tune_pick *picks, int64_t n);

/*
 * Learned cost model (16 -> 64 -> 64 -> 4 perceptron, ReLU hidden units):
 * from a group's 16 shape features (those of qtn_tune_rec) it predicts the
 * natural log of the launch time in milliseconds of each QTN_VAR_* variant.
 * Forward, backward and Adam run in FP32 HIP kernels on the caller's
 * stream; parameters live on the host between calls.  Parameter layout
 * (floats): W1[16][64], b1[64], W2[64][64], b2[64], W3[64][4], b3[4].
 */
#define QTN_MLP_PARAMS 5508
typedef struct qtn_costmodel qtn_costmodel;

/* A model with the given initial parameters (drawn by the caller). */
int qtn_costmodel_create(const float *params, qtn_costmodel **out);
int qtn_costmodel_params(const qtn_costmodel *cm, float *params_out);
/* Feature standardisation fixed by the first training call. */
int qtn_costmodel_normalization(const qtn_costmodel *cm, float *mean_out,
                                float *inv_std_out);
/* Device bytes for a batch of n samples. */
int qtn_costmodel_workspace(int64_t n, size_t *bytes_out);

/* Full-batch Adam (lr, beta1 0.9, beta2 0.999) for `epochs` steps on
 * features x[n][16] and times ms[n][4] (targets log ms; entries <= 0 are not
 * measured and carry no loss).  loss_history [epochs] or NULL. */
int qtn_costmodel_train(qtn_costmodel *cm, const float *x, const double *ms,
                        int64_t n, int32_t epochs, float lr, void *d_workspace,
                        size_t bytes, void *hip_stream, float *loss_history);

/* Predicted log-ms [n][4] for raw features x[n][16]. */
int qtn_costmodel_predict(const qtn_costmodel *cm, const float *x, int64_t n,
                          void *d_workspace, size_t bytes, void *hip_stream,
                          float *y_out);

/* Loss and gradient at the current parameters for inputs already
 * standardised (x[n][16]), targets t[n][4] and mask m[n][4]. */
int qtn_costmodel_grad(const qtn_costmodel *cm, const float *x, const float *t,
                       const float *m, int64_t n, void *d_workspace,
                       size_t bytes, void *hip_stream, float *loss_out,
                       float *grad_out);

/* One Adam step with a caller-given gradient. */
int qtn_costmodel_adam_step(qtn_costmodel *cm, const float *grad, float lr,
                            void *d_workspace, size_t bytes, void *hip_stream);

/* Picks, for every group of a planned network that the width rule gives its
 * own launch, the kernel with the lowest predicted time (the matrix form only
 * for complex64 groups that have one; QTN_VAR_STREAM runs as the cell mapping
 * where it fits, else the lane-sum streaming mapping) and rebuilds the
 * schedule; groups the rule places inside a workgroup stay there (counted as
 * QTN_VAR_BLOCK).
 * counts_out [4] or NULL: groups per QTN_VAR_*.  Workspace: the
 * cost-model bytes for as many samples as the network has groups. */
int qtn_apply_costmodel(qtn_network *net, const qtn_costmodel *cm,
                        void *d_workspace, size_t bytes, void *hip_stream,
                        int32_t *counts_out);

void qtn_costmodel_free(qtn_costmodel *cm);

/* Plan statistics. */
typedef struct qtn_plan_stats {
    int64_t n_buckets;    /* non-empty buckets over all light cones      */
    int64_t n_groups;     /* fused groups (= buckets when max_levels 1)  */
    int64_t n_wide;       /* groups launched one per kernel             */
    int32_t max_width;    /* widest bucket                               */
    int32_t width_hist[40]; /* buckets per width                         */
    double bytes;         /* algorithmic HBM bytes of one evaluation     */
    double flops;         /* complex-arithmetic FLOPs of one evaluation  */
    double paper_flops;   /* 8 * sum 2^width (the paper's Sec. II-E count) */
    size_t workspace;     /* device bytes                                 */
    int64_t n_matrix;     /* groups scheduled in matrix form (QTN_VAR_MFMA) */
    int64_t n_cell;       /* groups scheduled with the cell mapping        */
    int64_t n_stream;     /* groups scheduled with the streaming mapping,
                           * in own launches or inside workgroup segments */
    int64_t n_over4g;     /* groups with an operand larger than 4 GiB      */
    int64_t n_over4g_generic; /* of those, groups run by the generic mapping:
                           * all of them, as the streaming and cell mappings
                           * use 32-bit byte offsets within an operand     */
    int64_t n_sliced;     /* light cones planned with index slicing          */
    int64_t n_slices;     /* slices over all light cones (1 per unsliced one) */
} qtn_plan_stats;

int qtn_get_plan_stats(const qtn_network *net, qtn_plan_stats *out);

/* Variables of one light cone fixed by index slicing (slice bit k is
 * vars_out[k]); *n_out receives their count (0: not sliced).  vars_out holds
 * up to `cap` entries (10 suffice). */
int qtn_slice_vars(const qtn_network *net, int64_t edge, int32_t cap, int32_t *vars_out,
                   int32_t *n_out);

/* Width of each bucket of one light cone in the planned order, indexed by
 * elimination position (0 for an empty bucket).  widths_out [n_vars]. */
int qtn_bucket_widths(const qtn_network *net, int64_t edge, int32_t *widths_out);

void qtn_network_free(qtn_network *net);

/*
 * One bucket contraction of caller-given tensors (Sec. II-B: the tensors of a
 * bucket are multiplied over the union of their binary indices and the
 * bucket index is summed out; with several summed indices, the merged form of
 * Sec. II-C), with the kernels of the network path.  It isolates the bucket
 * kernel for synthetic contraction benchmarks (Sec. II-E, Tab. III).
 *
 * Indices are binary and named by int32 labels.  The summed labels are the
 * operand labels that out_labels does not list.  Union order: the summed
 * labels in ascending value, then out_labels in the order given.  A tensor
 * of rank r is a dense array of 2^r complex elements (complex128: two
 * doubles re, im; complex64: two floats) whose element-index bit j is its
 * j-th label: bit 0 is the least significant.  Each operand must list its
 * labels in union order (the layout bucket elimination stores tensors in).
 *   n_ops         1..64 operands
 *   ranks         [n_ops] ranks, 0..32
 *   labels        the operands' labels, concatenated ([sum ranks])
 *   offsets       [n_ops] byte offsets of the operands in the data buffer,
 *                 multiples of the element size
 *   n_out, out_labels, out_offset   the output tensor (rank n_out, its
 *                 labels, its byte offset); it may not overlap an operand
 *   precision     QTN_C128 or QTN_C64 (every tensor in that precision)
 *   variant       kernel mapping as qtn_config.variant: 0 the width rule,
 *                 1 generic, 2 streaming, 3 matrix form (operands that split
 *                 into two sides with at least 4 labels private to each), 4
 *                 cell mapping; a mapping that does not fit falls back to the
 *                 rule
 *   knob          streaming: lane-summed labels; cells: cell bits (2..4);
 *                 0 the default
 *   out           receives the plan (host memory, library-owned)
 * The summed count is 1..8 and the union holds at most 32 labels.
 * Errors: QTN_EINVAL (labels, offsets, ranks or overlap), QTN_ERANGE (more
 * than 8 summed labels, more than 32 in the union), QTN_ENOMEM.
 */
typedef struct qtn_bucket qtn_bucket;
int qtn_bucket_plan(int32_t n_ops, const int32_t *ranks, const int32_t *labels,
                    const int64_t *offsets, int32_t n_out, const int32_t *out_labels,
                    int64_t out_offset, int32_t precision, int32_t variant, int32_t knob,
                    qtn_bucket **out);

typedef struct qtn_bucket_info {
    int32_t w, L, n_ops;    /* union width, summed labels, operands          */
    int32_t variant;        /* mapping chosen: 0 generic, 1 streaming,
                               2 matrix form, 3 cells                        */
    int32_t knob, serial;   /* streaming: lane-summed labels; cells: cell
                               bits; serially walked summed labels           */
    int64_t n_units;        /* wave units (matrix form: output tiles)        */
    double bytes;           /* algorithmic HBM bytes (operands + output)     */
    double flops;           /* complex-arithmetic FLOPs                      */
    size_t workspace_bytes; /* device bytes of the descriptors               */
    int64_t data_bytes;     /* smallest data buffer holding every tensor     */
} qtn_bucket_info;

int qtn_bucket_get_info(const qtn_bucket *b, qtn_bucket_info *out);

/*
 * Run a planned bucket on the caller's stream (asynchronous: returns after
 * the launch is queued).
 *   d_data       device buffer holding the tensors at the planned offsets,
 *                at least data_bytes of qtn_bucket_get_info, 256-byte aligned
 *   d_workspace  device memory of at least workspace_bytes, 256-byte
 *                aligned; the descriptors are copied into it on the stream,
 *                so it must stay untouched until the kernel has run
 * Errors: QTN_EINVAL, QTN_ENOMEM (buffer or workspace too small),
 *         QTN_EDEVICE.
 */
int qtn_bucket_contract(const qtn_bucket *b, void *d_data, size_t data_bytes,
                        void *d_workspace, size_t ws_bytes, void *hip_stream);

/* qtn_bucket_contract with start and stop events attached to the kernel's
 * dispatch: blocks until the kernel has run and stores its duration in
 * milliseconds (the descriptor upload is not included). */
int qtn_bucket_contract_timed(qtn_bucket *b, void *d_data, size_t data_bytes,
                              void *d_workspace, size_t ws_bytes, void *hip_stream,
                              double *kernel_ms);

/*
 * qtn_bucket_contract without a workspace argument and without any device
 * allocation, for callers that cannot allocate device memory (tight serving
 * or benchmark loops, harnesses that forbid hipMalloc).  The descriptors go
 * into a fixed device array inside the library (16 KiB, one per GPU, held
 * until the process ends) instead of a caller workspace; nothing is
 * allocated or freed.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (on different streams, or from several threads)
 * race and must be serialised by the caller; calls on one stream are ordered.
 * Errors: QTN_ERANGE when the bucket's descriptors (workspace_bytes of
 * qtn_bucket_get_info) exceed 16 KiB; otherwise as qtn_bucket_contract.
 */
int qtn_bucket_contract_noalloc(const qtn_bucket *b, void *d_data, size_t data_bytes,
                                void *hip_stream);

void qtn_bucket_free(qtn_bucket *b);

const char *qtn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QTN_H */
