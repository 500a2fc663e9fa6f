/*
 * tn.h -- C interface of libtn, exact inference on probabilistic graphical
 * models by tensor-network contraction on one MI355X (gfx950).
 *
 * The library contracts the network of factor tensors of a model along a
 * binary contraction tree (paper: definition of a tensor network and
 * eq. contraction-definition; contraction orders as binary trees).  Each tree
 * node is one pairwise contraction executed by hand-written HIP kernels.
 *
 *   tn_logZ       probability of evidence / partition function (eq. pr),
 *   tn_marginals  all single-variable marginals (eq. mar-prob) through the
 *                 unity-vector adjoint pass (theorem thm:diff, eq. einback),
 *   tn_map        most probable explanation by max-plus contraction
 *                 (eq. tropical, eq. log-map) and argmax readout,
 *   tn_mmap       maximum marginal a posteriori by the two-phase method
 *                 (eq. mmap and the partition procedure after it),
 *   tn_sample     unbiased samples by back-tracing the tree (eq. sample,
 *                 eq. condition-prob).
 *
 * Conventions
 *   - Every call returns a tn_status; no C++ exception crosses this
 *     interface.  On a non-OK status the outputs are unspecified and
 *     tn_last_error() returns a thread-local message.
 *   - Input arrays are copied before the call returns; the caller keeps
 *     ownership.  Host outputs are caller-allocated.  Pointers named *_dev
 *     are device pointers owned by the caller (e.g. torch tensors); the
 *     library never frees them.
 *   - Variables are numbered 0..n_vars-1 with domain sizes card[v] >= 1.
 *     A factor's table is row-major over its scope in the order given,
 *     last variable fastest.
 *   - Evidence arrays hold one int32 per variable: -1 = unobserved,
 *     otherwise the observed value (0 <= e < card).
 *   - A plan owns device memory and one HIP stream (its own, or one the
 *     caller lends); calls on one plan are not re-entrant.  Different plans
 *     may be used from different threads.
 */
#ifndef TN_H
#define TN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_net tn_net;
typedef struct tn_plan_impl tn_plan_t;  /* created by tn_plan() */

typedef enum {
  TN_OK = 0,
  TN_E_INVALID = 1,        /* malformed input (message says which) */
  TN_E_NOMEM = 2,          /* host or device allocation failed */
  TN_E_DEVICE = 3,         /* a HIP call failed */
  TN_E_TOO_LARGE = 4,      /* an intermediate exceeds the size limits */
  TN_E_ZERO_EVIDENCE = 5,  /* p(e) = 0 for some instance */
  TN_E_UNSUPPORTED = 6     /* task not enabled in this plan / mode */
} tn_status;

typedef enum { TN_F32 = 0, TN_BF16 = 1, TN_F16 = 2 } tn_dtype;

/* Semiring bits for tn_plan_opts.semiring_mask. */
#define TN_SUM_PRODUCT 1   /* log Z, marginals, sampling */
#define TN_MAX_PLUS 2      /* MAP */

/* Evidence modes for tn_plan_opts.evidence_mode. */
#define TN_EVIDENCE_NONE 0       /* no evidence; batch must be 1 */
#define TN_EVIDENCE_SLICED 1     /* observed set fixed at plan time, values per
                                    call; factors are sliced (paper: the sliced
                                    tensor set of eq. pr) */
#define TN_EVIDENCE_INDICATOR 2  /* per-instance observed sets; every variable
                                    gets an indicator vector (one-hot when
                                    observed) and instances run as one batch */

/* Planner choices for tn_plan_opts.planner. */
#define TN_PLANNER_BEST 0        /* best of all strategies below */
#define TN_PLANNER_GREEDY 1      /* pairwise greedy on output size */
#define TN_PLANNER_MINFILL 2     /* bucket elimination, min-fill order */
#define TN_PLANNER_NATURAL 3     /* bucket elimination in variable-id order */
#define TN_PLANNER_MINDEG 4      /* bucket elimination, min-degree order */

typedef struct {
  int32_t semiring_mask;     /* TN_SUM_PRODUCT | TN_MAX_PLUS */
  int32_t evidence_mode;     /* TN_EVIDENCE_* */
  const int32_t *observed;   /* mode SLICED: observed variable ids */
  int32_t n_observed;
  const int32_t *query;      /* MMAP max variables (Q); NULL if no MMAP */
  int32_t n_query;
  int32_t planner;           /* TN_PLANNER_* */
  int32_t restarts;          /* randomised restarts per strategy */
  uint64_t seed;             /* planner tie-break seed */
  double max_log2_size;      /* slicing cap on log2(elements) of any
                                intermediate; 0 = no slicing.  MMAP plans
                                slice each group's sum; sum-product plans
                                (modes NONE / SLICED, no max-plus, no factor
                                gradients) slice the tree and then support
                                tn_logZ (Z summed over the slices) and
                                tn_sample (each sample ends in slice s with
                                probability Z_s / Z: one pass over the slices
                                in order, sample i taking slice s with
                                probability Z_s / (Z_0 + ... + Z_s)) */
  int32_t dtype;             /* tn_dtype of the matrix-core operands of the
                                sum-product contractions (dense form and fused
                                segments): TN_F32, or TN_BF16 / TN_F16 (operands
                                rounded to nearest, FP32 accumulation).  Every
                                stored tensor stays FP32 with its power-of-two
                                scale; the other kernels compute in FP32. */
  int32_t max_batch;         /* mode INDICATOR: instances per call */
  int32_t use_graph;         /* capture each task's launches in a hipGraph */
  void *hip_stream;          /* borrowed hipStream_t; NULL = library-owned */
  const int32_t *tree_pairs; /* optional precomputed contraction tree:
                                n_tree_pairs pairs (l, r) in post-order over
                                the leaf ids described at tn_plan() */
  int32_t n_tree_pairs;
  int32_t want_factor_grad;  /* keep factor adjoints (tn_logZ_dev grads) */
  int32_t host_only;         /* build host structures only (no device memory);
                                only tn_plan_info_get / tn_plan_tree / tn_free_plan
                                may then be called */
  int32_t no_fuse;           /* 0: fuse chains of small-operand contractions into
                                segments and run two consecutive segments of a
                                chain as one carrier pass where the tiles fit
                                (the intermediate carrier is never stored);
                                1: keep every tree node a separate contraction;
                                2: segments, one carrier pass each */
  int32_t autotune;          /* 1: at plan time, time every eligible kernel form
                                (generic, row, batch-uniform row, wave, dense) of each distinct
                                contraction shape on the device and keep the
                                fastest; 0: fixed rules.  The interleaved
                                layout's tile variants always follow rules. */
  int32_t batch_layout;      /* batched evidence (mode INDICATOR, max_batch > 1):
                                0 automatic (interleaved for dtype TN_F32),
                                1 instance-major (each instance's tensor
                                contiguous; all kernel forms, matrix cores),
                                2 interleaved (element e of instance b at
                                e * B + b with B = max_batch rounded up to a
                                multiple of 64: one wavefront computes one
                                output element for 64 instances, FP32 on the
                                vector ALUs) */
  const int64_t *joint_ptr;  /* joint marginals (tn_joint_marginals): n_joint + 1
                                offsets into joint_vars, set k = joint_vars
                                [joint_ptr[k], joint_ptr[k + 1]); NULL = none */
  const int32_t *joint_vars; /* variables of the sets (distinct within a set) */
  int32_t n_joint;           /* number of sets; each adds a unity tensor over
                                its variables to the network (leaf ids after
                                the unity vectors, in set order) */
} tn_plan_opts;

/* Summary of a plan (tn_plan_info). */
typedef struct {
  int32_t n_leaves, n_nodes;     /* main tree */
  int32_t n_kernels_fwd;         /* launches of one sum-product forward */
  int32_t n_kernels_bwd;         /* launches of the adjoint pass */
  int32_t n_kernels_max;         /* launches of the max-plus pass */
  double sc;                     /* log2 elements of the largest node output */
  double sc_union;               /* log2 of the largest node label union */
  double tc;                     /* log2 of sum over nodes of union sizes */
  double flops_fwd;              /* algorithmic flops of one sum-product
                                    forward: 2 x sum of union sizes, per instance */
  double bytes_fwd;              /* algorithmic bytes of one forward */
  int32_t n_sliced;              /* sliced labels */
  int32_t planner_used;          /* TN_PLANNER_* that won */
  int64_t device_bytes;          /* device memory held by the plan (host_only plans: the
                                    float arena it would allocate) */
  int32_t n_launches_fwd;        /* kernel launches after stage grouping */
  int32_t n_launches_bwd;
  int32_t n_launches_max;
  int32_t n_segments;            /* fused chain segments */
  int32_t n_fused_nodes;         /* tree nodes inside fused segments */
  int32_t n_dense;               /* contractions (forward and reverse) in the dense matrix-core form */
  int32_t n_wave;                /* contractions in the wave-per-output form (all passes, both semirings) */
  int32_t n_interleaved;         /* contractions in the interleaved-instance form */
  int32_t batch_stride;          /* interleaved plans: instances held per element (max_batch
                                    rounded up to a multiple of 64); 0 otherwise */
  int32_t n_dense_large;         /* of n_dense: contractions with 128 x 128 output tiles */
  int32_t two_front;             /* 1: the tree is the two-front variant of the planner's
                                    elimination order (two intermediates grown from both ends
                                    of the order, contracted side by side until they meet) */
  int32_t n_levels;              /* levels of the main tree (longest leaf-to-root path) */
  int32_t n_pairs;               /* pairs of consecutive segments run in one carrier pass */
  int32_t n_pairs_moved;         /* of n_pairs: pairs whose tiles take a common outer label
                                    into one map's rows and columns (that map applied as
                                    M (x) I over it) */
} tn_plan_info;

/* Fill *o with defaults: sum-product + max-plus, no evidence, best planner,
 * 4 restarts, no slicing, FP32, batch 1, graphs on, own stream. */
void tn_plan_opts_default(tn_plan_opts *o);

/*
 * Copy a factorised model.  scope_ptr has n_factors+1 entries (CSR into
 * scope_vars); values are concatenated per factor (row-major over the scope
 * order, last fastest), linear potentials >= 0 or, if values_are_log,
 * log-potentials (finite or -inf).  Scope variables of one factor must be
 * distinct.  Errors: TN_E_INVALID.
 */
tn_status tn_load_network(int32_t n_vars, const int32_t *card, int32_t n_factors,
                          const int64_t *scope_ptr, const int32_t *scope_vars,
                          const double *values, int32_t values_are_log, tn_net **out);
void tn_free_network(tn_net *net);

/*
 * A model file in the UAI inference-competition format (the format of the
 * problem sets of the paper's benchmarks): preamble MARKOV or BAYES, the
 * number of variables, their domain sizes, the number of functions, each
 * function's scope (size, then variable ids), then each function's table
 * (entry count, then the entries row-major over the scope, last variable
 * fastest; linear values).  White space of any kind separates tokens.  A
 * BAYES file's conditional probability tables load as factors unchanged.
 * Errors: TN_E_INVALID (unreadable file, malformed content; the message
 * names the file and the token), TN_E_NOMEM.
 */
tn_status tn_load_uai(const char *path, tn_net **out);

/*
 * A UAI evidence file: "n v_1 x_1 ... v_n x_n" (one evidence set) or a set
 * count m followed by m such sets.  Writes up to cap_rows rows of n_vars
 * int32 (-1 = unobserved) into evidence and the number of sets in the file
 * to *n_rows (call with cap_rows = 0 to size the buffer).  card (n_vars
 * entries) checks the values.  Errors: TN_E_INVALID.
 */
tn_status tn_read_uai_evidence(const char *path, int32_t n_vars, const int32_t *card, int32_t *evidence,
                               int32_t cap_rows, int32_t *n_rows);

/* A UAI query file "n q_1 ... q_n" (e.g. the MMAP max variables): writes up
 * to cap ids to vars and n to *n.  Errors: TN_E_INVALID. */
tn_status tn_read_uai_query(const char *path, int32_t n_vars, int32_t *vars, int32_t cap, int32_t *n);

/* Read back a loaded network: sizes (any pointer may be NULL), then the
 * arrays in the layout of tn_load_network (caller-allocated; NULL skips). */
tn_status tn_network_sizes(const tn_net *net, int32_t *n_vars, int32_t *n_factors, int64_t *n_scope,
                           int64_t *n_values);
tn_status tn_network_get(const tn_net *net, int32_t *card, int64_t *scope_ptr, int32_t *scope_vars,
                         double *values, int32_t *values_are_log);

/*
 * Build a plan: leaves, contraction tree, per-node kernel descriptors,
 * device buffers.  Leaf ids (for tree_pairs): factors 0..n_factors-1 in
 * load order, then one unity vector per variable in increasing id order --
 * all variables for modes NONE and INDICATOR, only unobserved ones for mode
 * SLICED -- then one unity tensor per joint set (joint_*), in set order
 * (none for a set whose variables are all observed in mode SLICED).
 * (paper: MAR algorithm step 1 adds one unity tensor per query variable;
 * with batched evidence it doubles as the evidence indicator.)
 * With a query set, the plan holds the two MMAP phases instead.
 * Errors: TN_E_INVALID (bad options or tree), TN_E_TOO_LARGE, TN_E_NOMEM,
 * TN_E_DEVICE.
 */
tn_status tn_plan(const tn_net *net, const tn_plan_opts *opts, tn_plan_t **out);
void tn_free_plan(tn_plan_t *plan);
tn_status tn_plan_info_get(const tn_plan_t *plan, tn_plan_info *info);

/* Copy the main contraction tree: writes up to cap pairs (post-order) and
 * returns the count in *n_pairs and the leaf count in *n_leaves. */
tn_status tn_plan_tree(const tn_plan_t *plan, int32_t *pairs, int32_t cap, int32_t *n_pairs,
                       int32_t *n_leaves);

/* Sliced variables of a plan (ascending; slices enumerate their values in
 * row-major order, last fastest): writes up to cap ids, *n = count. */
tn_status tn_plan_sliced(const tn_plan_t *plan, int32_t *vars, int32_t cap, int32_t *n);

/*
 * Planning only (host, no device): contraction tree and complexity of the
 * network under the given options, for inspection and testing.
 * pairs: caller buffer of at least 2*(n_leaves-1) int32 (n_leaves as
 * described at tn_plan); stats: optional.
 */
tn_status tn_plan_tree_host(const tn_net *net, const tn_plan_opts *opts, int32_t *pairs,
                            int32_t cap, int32_t *n_pairs, int32_t *n_leaves,
                            tn_plan_info *stats);

/*
 * log p(e) per instance (eq. pr).  evidence: [batch][n_vars] (may be NULL
 * for mode NONE).  batch: 1 for modes NONE/SLICED (SLICED may pass several
 * instances; they run one after another), <= max_batch for INDICATOR.
 * logz: [batch] FP64.  TN_E_ZERO_EVIDENCE if some p(e) = 0.
 */
tn_status tn_logZ(tn_plan_t *plan, int32_t batch, const int32_t *evidence, double *logz);

/*
 * log p(e) and p(v = x | e) for every variable (eq. mar-prob via the
 * adjoint pass of theorem thm:diff).  marg: [batch][sum_v card[v]] FP64,
 * variable-major; observed variables get a one-hot row.
 */
tn_status tn_marginals(tn_plan_t *plan, int32_t batch, const int32_t *evidence, double *logz,
                       double *marg);

/*
 * Joint marginals p(x_S | e) of the plan's variable sets (tn_plan_opts
 * joint_*): the adjoint of a unity tensor over each set, normalised (the MAR
 * algorithm's unity tensors over several variables; theorem thm:diff).
 * joint: [batch][sum_k prod_{v in S_k} card[v]] FP64; set k's table is
 * row-major over its variables sorted ascending (last fastest), zero where an
 * observed variable takes another value.  logz optional.  Modes as for
 * tn_marginals.  TN_E_UNSUPPORTED if the plan has no sets.
 */
tn_status tn_joint_marginals(tn_plan_t *plan, int32_t batch, const int32_t *evidence, double *logz,
                             double *joint);

/*
 * Factor marginals p(x_f | e) = T_f(x_f) Tbar_f(x_f) / Z for every factor
 * (theorem thm:diff: Tbar_f = dZ / dT_f, and the products sum to Z over the
 * factor's scope).  fmarg: [batch][n_values] FP64, laid out as the values of
 * tn_load_network (scope order as loaded, last fastest), zero where an
 * observed variable takes another value.  logz optional.  Needs a plan built
 * with want_factor_grad; modes as for tn_marginals.
 */
tn_status tn_factor_marginals(tn_plan_t *plan, int32_t batch, const int32_t *evidence, double *logz,
                              double *fmarg);

/*
 * MPE (eq. log-map): assign [batch][n_vars] (evidence copied in), logp
 * [batch] = max log p(x, e) as computed in FP32.  Ties keep the smallest
 * row-major index over each node's eliminated variables (sorted by id).
 */
tn_status tn_map(tn_plan_t *plan, int32_t batch, const int32_t *evidence, int32_t *assign,
                 double *logp);

/*
 * MMAP (eq. mmap) for the plan's query set: assign_q [n_query] in the
 * order of the sorted query ids, log_value = max_q log sum_m p(q, m, e)
 * (optional: NULL skips it).  TN_E_ZERO_EVIDENCE if p(e) = 0.
 */
tn_status tn_mmap(tn_plan_t *plan, const int32_t *evidence, int32_t *assign_q, double *log_value);

/*
 * n samples from p(x | e) (eq. sample / eq. condition-prob), Philox4x32-10
 * uniforms with key = seed and counter (sample, node, slot).
 * samples: [n][n_vars].
 */
tn_status tn_sample(tn_plan_t *plan, const int32_t *evidence, int64_t n, uint64_t seed,
                    int32_t *samples);

/*
 * tn_sample for callers that cannot allocate device memory (code that must
 * not call hipMalloc: serving loops, harnesses that forbid allocation, work
 * issued around stream capture).  Same arguments, results and Philox stream
 * as tn_sample; the device staging of the samples (rows, and on sliced plans
 * the ids of the samples drawn in one slice) lives in a static array of
 * 2^22 int32 (16 MiB) that the library holds on each GPU until the process
 * ends, instead of plan memory grown on demand.  The call launches kernels
 * directly (no graph capture or instantiation) and allocates nothing on the
 * device.  Limit: n * n_vars (+ 2 n + 64 on sliced plans) <= 2^22, else
 * TN_E_TOO_LARGE.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (several threads or plans at once) race and must be
 * serialised by the caller.
 */
tn_status tn_sample_noalloc(tn_plan_t *plan, const int32_t *evidence, int64_t n, uint64_t seed,
                            int32_t *samples);

/*
 * Device-side sum-product for differentiation (theorem thm:diff): factor
 * tables come from values_dev (FP32, linear, laid out as in
 * tn_load_network), log Z goes to logz_dev (FP64, one value), and if
 * grad_dev is not NULL it receives d logZ / d T_f for every factor entry
 * (FP32, same layout; requires want_factor_grad).  Modes NONE and SLICED
 * (evidence as in tn_logZ, one instance).  Runs on the plan's stream.
 */
tn_status tn_logZ_dev(tn_plan_t *plan, const int32_t *evidence, const float *values_dev,
                      double *logz_dev, float *grad_dev);

/* Per-launch timing of one task (for roofline reports).  kind: 0/1 generic
 * contraction (sum / max), 2/3 split-reduction contraction (sum / max),
 * 4 leaf preparation, 5 other, and the kernels of fused chain segments:
 * 6 carrier forward (C_L = M C_0 over the outer labels), 7 carrier reverse
 * (adjoint of C_0 and partial sums of Gbar C_0^T), 8 composed maps M of a
 * stage's segments, 9 adjoint sweeps (small operands' adjoints) of a
 * stage's segments, 10 dense-form contractions on the matrix cores
 * (sum-product), 11 dense-form max-plus contractions (vector ALUs),
 * 12 / 13 interleaved-form contractions (sum / max).  flops and bytes are algorithmic: 2 x output x summed
 * elements; 4 bytes x (|X| + |Y| + |Z|) per instance times the instances of
 * the launch; for a carrier forward 4 bytes x (|input carrier| + |output
 * carrier|), for a carrier reverse 4 bytes x (2 |input carrier| + |output
 * carrier|) (it reads the input carrier and the output's adjoint and writes
 * the input's adjoint).  ms is the launch's duration from HIP events
 * recorded around it on the plan's stream, averaged over reps. */
typedef struct {
  int32_t kind;
  double flops, bytes, ms;
} tn_op_profile;

/* task: 0 log Z, 1 log Z + marginals, 2 MAP, 3 (MMAP plans) the sum phase of
 * every group for its first slice (sliced variables at 0; evidence one row;
 * batch ignored).  Runs the task reps times
 * without graph capture and fills out[0..min(cap, n)-1]; *n_ops = n. */
tn_status tn_profile(tn_plan_t *plan, int32_t task, int32_t batch, const int32_t *evidence,
                     int32_t reps, tn_op_profile *out, int32_t cap, int32_t *n_ops);

/* Average over the launches of one kind of one task, timed back to back
 * (all launches of that kind in task order, reps times) between two HIP
 * events on the plan's stream: avg->ms per launch, avg->flops and
 * avg->bytes per launch; *n_launches = launches of that kind per task. */
tn_status tn_profile_kind(tn_plan_t *plan, int32_t task, int32_t kind, int32_t batch,
                          const int32_t *evidence, int32_t reps, tn_op_profile *avg,
                          int32_t *n_launches);

/*
 * Autotuner decisions.  A plan built with autotune = 1 times the eligible
 * kernel forms of each distinct contraction shape once per process and GPU
 * architecture; later plans with the same shape reuse the decision, so two
 * plans of one model in one process run the same kernels and give
 * bit-identical results (the forms sum in different orders).
 *   tn_tune_save  writes every decision held by the process to a text file
 *                 (one line each); *n_saved (optional) = their count.
 *   tn_tune_load  reads such a file and adds its decisions (replacing held
 *                 ones for the same shape); plans built afterwards use them
 *                 instead of timing.  TN_E_INVALID if the file cannot be read
 *                 or is malformed (then nothing is added).
 *   tn_tune_clear forgets every decision.
 * Thread-safe; no device work.
 */
tn_status tn_tune_save(const char *path, int64_t *n_saved);
tn_status tn_tune_load(const char *path, int64_t *n_loaded);
void tn_tune_clear(void);

/* Contractions of one task, for inspection: per contraction its kernel form
 * (0 generic one lane per output, 1 row (variant 1: one batch assignment per
 * wavefront, Y's block of it read once per wavefront), 2 dense on the matrix cores or, for
 * max-plus, the vector ALUs, 3 wave per output, 4 interleaved instances, 5
 * fused-segment kernel with variant 1 carrier pass, 2 its reverse, 3
 * composed maps, 4 adjoint sweeps, 5 carrier pass of two consecutive
 * segments, 6 its reverse), semiring (0 sum-product, 1 max-plus), the label
 * classes' sizes (rows = output labels held by X, columns = output labels X
 * lacks, summed = labels of X or Y not in the output) and the operands'
 * elements per instance.  task: 0 forward sum-product (fused list when the
 * plan fuses), 1 reverse pass, 2 max-plus, 3 MMAP plans: the sum phase of
 * every group.  Writes up to cap entries; *n = count. */
typedef struct {
  int32_t form, semiring, variant;   /* variant: tile / order variant of the form */
  int64_t rows, cols, summed;
  int64_t x_size, y_size, z_size;
  int32_t eligible;                  /* forms the autotuner may choose among (bits: 1 generic,
                                        2 row, 4 dense, 8 wave, 16/32/64/128 interleaved tiles,
                                        256 dense 128 x 128 tiles, 512 generic in output order,
                                        1024 batch-uniform row); 0 for fused-segment kernels */
} tn_op_info;
tn_status tn_plan_ops(const tn_plan_t *plan, int32_t task, tn_op_info *out, int32_t cap, int32_t *n);

/* Synchronise the plan's stream; TN_E_DEVICE on error. */
tn_status tn_sync(tn_plan_t *plan);

/* Thread-local message for the last non-OK status. */
const char *tn_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TN_H */
