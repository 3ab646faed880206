/*
 * pa.h -- C ABI of the MI355X (gfx950) pixel array library, libpa.so.
 *
 * The pixel array method (Spivak, Dobson, Kumari, Wu, arXiv 1609.00061)
 * solves a system of relations on a bounding box for a chosen set of exposed
 * variables:
 *   1. every relation R_i is plotted as a Boolean array over the pixels of its
 *      variables (Sec. 3.2, "Plotting relations as arrays"; the pixel grid is
 *      eqn Pixel_def: resolution r cuts [a, b) into r pixels of width
 *      (b - a) / r);
 *   2. the plots are combined by generalized array multiplication
 *      (Sec. 3.3, Alg. "Generalized array multiplication", eqn GAM):
 *      A'(e') = OR over link entries e with Entr'(e) = e' of AND_i A_i(e_i),
 *      i.e. latent variables are projected out by OR-of-ANDs;
 *   3. by associativity (Thm "associative") the multiplication is evaluated
 *      as a cluster tree (Sec. 3.5) of pairwise contractions.
 *
 * Plotting rule of this library: a relation f(vars) = 0 is evaluated at the
 * pixel corners x_k = a + k*delta (k = 0..r) and a pixel (a closed cell) is
 * set iff among its 2^n corners one has f <= 0 and one has f >= 0 (a corner
 * where f is NaN counts as neither).  The paper permits any sufficiently fast
 * and accurate plotting method (Sec. 3.6).  The sign of f at a corner is the
 * sign of a canonical FP64 value: nested Horner with correctly rounded fma in
 * the relation's declared variable order (last variable outermost), i.e.
 *   f = sum_i A_i(x_0..x_{n-2}) x_{n-1}^i,  p = A_d, p = fma(p, x_{n-1}, A_i),
 * every A_i evaluated by the same rule one variable down.  With
 * PA_PLOT_FP32_ESCALATE the corners are evaluated in FP32 first and only
 * corners whose |f| does not exceed a rigorous FP32 error bound are
 * re-evaluated canonically in FP64, so the result is bit-identical to
 * PA_PLOT_FP64.
 *
 * ------------------------------------------------------------------------
 * Bit-array layout (pa_bitarray).  An n-dimensional Boolean array with dims
 * d_0..d_{n-1} is stored row-major; the LAST axis is bit-packed LSB-first into
 * 32-bit words and every row of the last axis occupies `row_words` words,
 * which must equal pa_row_words(d_{n-1}) = 2 * ceil(d_{n-1} / 64) (rows are
 * padded to 64 bits).  Element (i_0..i_{n-1}) is bit (i_{n-1} % 32) of word
 *   ((i_0 * d_1 + i_1) * ... * d_{n-2} + i_{n-2}) * row_words + i_{n-1} / 32.
 * Padding bits must be zero in inputs and are zero in outputs.  A 0-dim
 * array is one word whose bit 0 is the value ("has a solution in the box",
 * fn. to Def. "entries").  `data` is a DEVICE pointer owned by the caller.
 *
 * Ownership and streams.  Host arrays passed in (axes, coefficients,
 * variable lists) are read during the call only.  Device buffers (outputs,
 * optional workspace) belong to the caller.  Work is enqueued on `stream`
 * (a hipStream_t; NULL means the default stream); calls that fill a
 * pa_report synchronize `stream` before returning.  A plan may be executed
 * repeatedly; executing one plan concurrently on two streams is a race
 * (its workspace is shared).
 *
 * Errors.  Every entry point returns a pa_status; nothing throws across the
 * ABI.  pa_last_error() returns a thread-local message for the last failure.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PA_MAX_DIMS 12        /* max rank of any array handled */
#define PA_MAX_ARITY 3        /* max variables of one relation */
#define PA_MAX_DEGREE 4       /* max total degree of a relation */
#define PA_MAX_VARS 64        /* max variables of one system */
#define PA_MAX_RELATIONS 32   /* max relations of one system */

typedef enum {
    PA_OK = 0,
    PA_EINVAL = 1,            /* invalid argument (see each entry point)          */
    PA_ENOMEM = 2,            /* workspace too small, allocation or size cap hit  */
    PA_EHIP = 3,              /* HIP runtime error (no device, launch failure...) */
    PA_EUNSUPPORTED = 4       /* valid but outside what the library implements    */
} pa_status;

/* One variable's discretization: a port's bounds and resolution
 * (Def. "pack"): range [lo, hi] with lo <= hi, resolution res >= 2. */
typedef struct {
    double lo, hi;
    int32_t res;
    int32_t reserved;
} pa_axis;

/* Target subset of a relation's defining function (Def.
 * "functionally_defined": the relations f = 0, f <= 0 and f < 0). */
enum { PA_TARGET_EQ = 0, PA_TARGET_LE = 1, PA_TARGET_LT = 2 };

/* A polynomial relation f(x_{vars[0]}, ..., x_{vars[arity-1]}) in S, with S
 * the target subset: {0}, (-inf, 0] or (-inf, 0).
 * coef has C(arity + degree, degree) entries in graded-lex order of the
 * monomials in the declared variable order: total degree ascending, then
 * lexicographically descending exponent tuples (for (x, y), degree 3:
 * 1, x, y, x^2, xy, y^2, x^3, x^2y, xy^2, y^3).  vars are distinct. */
typedef struct {
    int32_t arity;            /* 1..PA_MAX_ARITY  */
    int32_t degree;           /* 0..PA_MAX_DEGREE */
    const int32_t *vars;      /* host, arity entries, ids in [0, n_vars) */
    const double *coef;       /* host                                     */
    int32_t target;           /* PA_TARGET_* (0: f = 0)                   */
    int32_t reserved;         /* 0                                        */
} pa_relation;

/* Bit-packed Boolean array, layout above.  data is a device pointer. */
typedef struct {
    void *data;
    int32_t ndim;
    int32_t dims[PA_MAX_DIMS];
    int64_t row_words;
} pa_bitarray;

/* A system: the inner packs (relations) of a wiring diagram (Def. "wd") over
 * n_vars links; every variable must occur in some relation. */
typedef struct {
    int32_t n_vars;
    const pa_axis *axes;      /* host, n_vars entries */
    int32_t n_rel;
    const pa_relation *rel;   /* host, n_rel entries  */
} pa_system;

enum { PA_ORDER_GREEDY = 0, PA_ORDER_EXHAUSTIVE = 1, PA_ORDER_LEARNED = 2, PA_ORDER_GIVEN = 3 };
enum { PA_PLOT_FP32_ESCALATE = 0, PA_PLOT_FP64 = 1 };
/* Plotting rule (pa_opts.plot_rule).
 * PA_RULE_CORNER: f is evaluated at the pixel corners; for f = 0 a pixel is
 *   set iff one corner has f <= 0 and one has f >= 0, for f <= 0 (f < 0) iff
 *   one corner has f <= 0 (f < 0).
 * PA_RULE_CENTER: the epsilon-tolerance sample-in-center plot (Def.
 *   "sample_in_center", Cor. "guarantees"): f is evaluated at the pixel
 *   centre c_k = a + (k + 1/2) * delta (FP64, each operation rounded once) and
 *   a pixel is set iff the distance from f(c) to the target subset is at most
 *   eps = pa_opts.tolerance: |f(c)| <= eps, f(c) <= eps or f(c) < eps for the
 *   three targets.  With eps a valid tolerance (Sec. 3.2: f moves by less
 *   than eps within a pixel radius) the plot is eps-accurate, and so is the
 *   solution (Thm "extended").
 * Both rules decide with the canonical FP64 value (below); FP32 with
 * escalation gives the same bits. */
enum { PA_RULE_CORNER = 0, PA_RULE_CENTER = 1 };

typedef struct pa_model pa_model;   /* learned contraction-order cost model */

typedef struct {
    int32_t order_policy;     /* PA_ORDER_*                                         */
    int32_t n_given;          /* PA_ORDER_GIVEN: number of merges (n_rel - 1)       */
    const int32_t *given;     /* PA_ORDER_GIVEN: 2*n_given factor ids; relations are
                                 factors 0..n_rel-1 and merge t creates factor
                                 n_rel + t from the two listed factors             */
    int32_t precision;        /* PA_PLOT_*                                          */
    int32_t audit;            /* 1: also evaluate every corner in FP64 and count
                                 FP32/FP64 sign disagreements (slow; diagnostics)  */
    int32_t timing;           /* 1: time plot and contraction phases with events;
                                 2: also time every op (see pa_plan_op_times)       */
    int32_t plain;            /* 1: the plain GPU path: one kernel launch per relation
                                 plot and per contraction step, default tiles      */
    int32_t per_op;           /* 1: one launch per step like the plain path, but
                                 with all plots in one launch and split K         */
    int32_t graph;            /* 1: capture the executor's launches in a hipGraph on
                                 the first execute on a non-NULL stream with a
                                 given output buffer, and replay it afterwards     */
    int32_t single_launch;    /* 1: run the whole plan as ONE persistent launch whose
                                 tiles wait on per-step dependency counters; 0
                                 (default): one grouped launch per level of the
                                 cluster tree and step kind, across all steps      */
    int32_t persist_wg;       /* persistent workgroups (0: autotuned default)        */
    int32_t plot_strip;       /* cells walked per plot thread (0: default)           */
    int32_t contract_units;   /* output bits per streaming tile (0: default)         */
    const pa_model *model;    /* PA_ORDER_LEARNED: the cost model                   */
    void *workspace;          /* optional device workspace (NULL: library-owned)    */
    size_t workspace_bytes;
    int32_t autotune;         /* 1: pa_plan_create / pa_batch_create take the executor
                                 settings (single_launch, persist_wg, plot_strip,
                                 contract_units) from the autotuner: cached per
                                 workload structure and GPU architecture, tuned by
                                 timing on the device (stream 0) on a cache miss */
    int32_t gemm_split;       /* MFMA contractions: those of one tree level (one
                                 grouped launch) split their K range until the
                                 launch holds about this many work items (output
                                 tiles x parts); partial products are OR-ed into a
                                 zeroed output (exact); 1: never split; 0: default
                                 (512)                                            */
    int32_t gemm_path;        /* MFMA contractions: 1 = K chunks staged in LDS by the
                                 workgroup, 128x128 output tiles; 2 = each wave loads
                                 its own rows straight into registers (no LDS, no
                                 barriers); 3 = staged in LDS, 256x128 output tiles
                                 (4x2 MFMA blocks per wave); 4 = 256x128 tiles with
                                 the A operands kept in registers while consecutive
                                 tiles share their rows (K of at most 256 bits, else
                                 3); 0: default (4, or 3 when K is longer, for
                                 contractions of at least 8192 128x128 tiles, else
                                 1).  A single persistent launch (single_launch)
                                 uses 1 in place of 3, 4 and of the default     */
    int32_t verify_order;     /* PA_ORDER_LEARNED, pa_plan_create: 1 = when the model's
                                 tree differs from the exhaustive one, build both,
                                 time each on the device (one untimed and two timed
                                 executions on stream 0, temporary outputs) and keep
                                 the faster; the exhaustive search stays the judge */
    int32_t sparse_pass;      /* MFMA contractions whose B operand is a plotted
                                 relation get a sparse pass: the relation is also
                                 plotted with its output variables packed, and each
                                 output row is computed as the OR of the rows of
                                 that plot selected by the set bits of the A row.
                                 0 (default): contractions of at least 2^32 MACs
                                 get the pass with an MFMA fallback (a count step
                                 adds up the set bits of A; with at most
                                 sparse_max_density set bits per 1024 the pass
                                 computes the output and the MFMA kernel exits at
                                 once, otherwise the reverse).  1 = the pass with
                                 the fallback for every such contraction, 2 = the
                                 pass alone (no count, no MFMA kernel; B's first
                                 plot is dropped when nothing else reads it) for
                                 every such contraction, 3 = as 2, and two passes
                                 read only by one streamed contraction (output
                                 out[p][q] = OR over s, t of X[q][s][p][t] AND
                                 Y[p][s][q][t], t packed and at most 256 bits)
                                 are fused with it: lists of the set bits of the
                                 A operands, then one step that gathers the rows
                                 of both plots in LDS; the pass outputs are never
                                 stored.  -1 = never.  Not used by the plain path
                                 or a single persistent launch.                  */
    int32_t sparse_max_density; /* 0..1024 set bits per 1024 bits of A (0: 64)     */
    int32_t plot_rule;        /* PA_RULE_* (0: corners)                           */
    int32_t measure_density;  /* 1: plan creation plots every relation once on the
                                 device and counts its set cells; the learned
                                 order's density features (and those of
                                 pa_plan_step_samples) then start from these
                                 measured plot densities instead of an
                                 analytic estimate                               */
    double tolerance;         /* PA_RULE_CENTER: eps >= 0, finite                  */
} pa_opts;

typedef struct {
    int64_t corners;                       /* corners evaluated                            */
    int64_t corners_flagged;               /* corners escalated to FP64                    */
    int64_t corners_disagree;              /* audit: sign(FP32) != sign(FP64), all corners */
    int64_t corners_disagree_unflagged;    /* audit: same among non-escalated corners (0)  */
    int64_t nnz_out;                       /* set bits of the output                       */
    int32_t n_steps;                       /* pairwise contractions executed               */
    int32_t n_launches;                    /* kernel launches enqueued                     */
    int32_t merges[2 * PA_MAX_RELATIONS];  /* the chosen clustering, PA_ORDER_GIVEN format */
    double cost_macs;                      /* sum over steps of the product of the
                                              resolutions of the step's links
                                              (eqn naive_cost)                            */
    double t_plot_ms, t_contract_ms, t_plan_ms;
} pa_report;

typedef struct pa_plan pa_plan;

/* 2 * ceil(d / 64): words per row of a last axis of length d (d >= 1). */
int64_t pa_row_words(int32_t d);
/* Total words of an array with the given dims (1 for ndim == 0). */
int64_t pa_array_words(int32_t ndim, const int32_t *dims);

/* Plot one relation (Sec. 3.2) on the pixel grid of its variables.
 * axes_of_vars[j] is the discretization of the relation's j-th variable.
 * out: dims = (res of vars[0], ..., res of vars[arity-1]), the declared order.
 * EINVAL: arity/degree out of range, res < 2, lo > hi, non-finite bounds,
 * repeated variable, out dims or row_words mismatching.  report may be NULL. */
int pa_plot_relation(const pa_relation *rel, const pa_axis *axes_of_vars, const pa_opts *opts,
                     pa_bitarray *out, pa_report *report, void *stream);

/* Generalized array multiplication of two packs (eqn GAM with two inner
 * packs): C(out_vars) = OR over every variable of A or B not in out_vars of
 * A(a_vars) AND B(b_vars).  Variable ids are arbitrary labels in
 * [0, PA_MAX_VARS); a variable shared by A and B must have the same length in
 * both.  out_vars lists distinct variables of A or B, in C's axis order.
 * B may be NULL (then b_vars is ignored: a projection/permutation of A).
 * EINVAL on rank, dims, row_words or label mismatch; ENOMEM if the internal
 * workspace cannot be allocated. */
int pa_contract(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B, const int32_t *b_vars,
                const int32_t *out_vars, int32_t n_out, pa_bitarray *C, const pa_opts *opts, void *stream);

/* pa_contract for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, layouts and results, and no hipMalloc, hipFree or other
 * allocation.  Its one scratch buffer -- the latent-entry table of a streamed
 * contraction -- is a static device array of the library (1 MiB per GPU, kept
 * until the process ends), written by a kernel on `stream`; contractions with
 * more than 65536 latent entries (outside the packed latent variable) are
 * refused with PA_ENOMEM.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race. */
int pa_contract_noalloc(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B, const int32_t *b_vars,
                        const int32_t *out_vars, int32_t n_out, pa_bitarray *C, const pa_opts *opts, void *stream);

/* Generalized array multiplication of two Boolean packs in the semiring N of
 * natural numbers (the semiring footnote of Sec. 2.2; Notation, Ch. 3: the
 * method works over any semiring): C(out_vars) = the number of entries of the
 * variables of A or B not in out_vars at which A and B are both set -- the
 * density of solutions per pixel instead of their existence.  A, B, a_vars,
 * b_vars, out_vars as for pa_contract (B may be NULL: C counts A's set
 * entries over the other variables).  C: device, caller-owned, uint32 per
 * entry, row-major over out_vars with no padding (one entry for n_out = 0).
 * Counts are exact: EUNSUPPORTED when the latent variables have 2^31 or more
 * entries.  Canonical layouts (A = [batch][m][k], B = [batch][n][k],
 * C = [batch][m][n], as for the MFMA path of pa_contract) run on int8 MFMA
 * with 0/1 operands and int32 accumulation; others visit every latent entry
 * per output entry.  EINVAL as for pa_contract. */
int pa_contract_count(const pa_bitarray *A, const int32_t *a_vars, const pa_bitarray *B, const int32_t *b_vars,
                      const int32_t *out_vars, int32_t n_out, uint32_t *C, const pa_opts *opts, void *stream);

/* Plan a whole solve: choose the cluster tree (opts->order_policy), lay out
 * every intermediate, upload coefficient and axis tables and size the
 * workspace.  exposed lists the outer pack's variables in the output's axis
 * order (n_exposed may be 0: one-bit output).  EINVAL: invalid system (as for
 * pa_plot_relation, plus variable in no relation, exposed repeated or out of
 * range, n_rel > PA_MAX_RELATIONS); ENOMEM: workspace or intermediate size
 * cap exceeded. */
int pa_plan_create(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts *opts,
                   pa_plan **plan);
/* Enqueue the plotting and all contractions; out dims = resolutions of the
 * exposed variables in the given order.  report (may be NULL) is filled after
 * synchronizing the stream. */
int pa_plan_execute(pa_plan *plan, pa_bitarray *out, pa_report *report, void *stream);
/* Device bytes of the plan's workspace (intermediates + tables). */
size_t pa_plan_workspace_bytes(const pa_plan *plan);
/* JSON description of the plan (steps, kernels, layouts, costs) into buf;
 * returns the length needed (excluding the NUL). Host-only except under
 * PA_ORDER_LEARNED, whose model inference runs on the model's device, and
 * with opts->measure_density, whose plots run on the current device. */
int64_t pa_plan_describe(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts *opts,
                         char *buf, int64_t buf_len);
void pa_plan_destroy(pa_plan *plan);

/* Per-op kernel durations of the last pa_plan_execute of a plan created with
 * opts->timing == 2, measured with HIP events recorded on the execution
 * stream around each op (the persistent executor is one op of kind
 * PA_OPKIND_PERSIST whose macs are the plan's total).  Fills up to cap entries: ms[i] (milliseconds),
 * kind[i] (PA_OPKIND_*) and macs[i] (product of the op's link resolutions,
 * eqn naive_cost; 0 for plots and fills).  Waits for the events.  Returns
 * the number of ops, or -1 if the plan does not record op timings. */
enum { PA_OPKIND_BITS = 0, PA_OPKIND_STREAM_K = 1, PA_OPKIND_STREAM_W = 2, PA_OPKIND_GEMM = 10,
       PA_OPKIND_FILL = 20, PA_OPKIND_GATHER = 25, PA_OPKIND_COUNT = 26, PA_OPKIND_ROWLIST = 27, PA_OPKIND_FUSED = 28,
       PA_OPKIND_PLOT = 30, PA_OPKIND_PERSIST = 40 };
int32_t pa_plan_op_times(pa_plan *plan, double *ms, int32_t *kind, double *macs, int32_t cap);

/* Kernel duration of every grouped launch of a plan on the default
 * (level-grouped) executor, after at least one pa_plan_execute: for each
 * group in order, reps back-to-back launches of that group on `stream`
 * between two HIP events; ms[i] = elapsed / reps (so it includes the
 * dispatch gap between consecutive launches, not the event overhead of a
 * single launch).  Every group is idempotent given its inputs, so the
 * plan's output is unchanged; the plot flag counters accumulate.  kind[i]
 * and macs[i] as for pa_plan_op_times.  Synchronizes.  Returns the number of
 * groups, or -1 (see pa_last_error). */
int32_t pa_plan_time_groups(pa_plan *plan, int32_t reps, double *ms, int32_t *kind, double *macs, int32_t cap,
                            void *stream);
/* Bound of each dependency wait of the single persistent launch
 * (opts->single_launch), in polls of the producer step's done counter: 2^26
 * by default (seconds of waiting; the waits end well before in any correct
 * plan); a negative value makes every wait give up at its first poll.  A wait
 * that gives up makes every workgroup leave the launch (the kernel ends
 * normally, the output is incomplete), and the execute call that asks for a
 * report (pa_plan_execute with rep, pa_batch_execute with a report) returns
 * PA_EHIP, "persistent executor gave up a dependency wait".  For tests of that
 * failure path.  Waits for every call in flight on the device, then writes
 * the bound into the plan's device state (it holds for later executes).
 * Returns PA_OK, PA_EINVAL (null plan) or PA_EHIP. */
int pa_plan_set_wait_limit(pa_plan *plan, int64_t polls);

/* ---------------------------------------------------------- batches
 * Many independent systems solved together: each is planned on its own, all
 * share one workspace, and their steps are merged into one table sorted by
 * tree level and kind, so every grouped launch (or the single persistent
 * launch, opts->single_launch) works on tiles of many systems at once; with
 * opts->graph the whole batch is one hipGraph replay.  exposed[i] /
 * n_exposed[i] describe system i's outer pack.  opts->plain and opts->per_op
 * are not accepted (EINVAL).  EINVAL/ENOMEM as for pa_plan_create, with the
 * failing system's index in pa_last_error(). */
typedef struct pa_batch pa_batch;
int pa_batch_create(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed,
                    const int32_t *n_exposed, const pa_opts *opts, pa_batch **batch);
/* outs[i]: system i's output (dims = its exposed resolutions).  report (the
 * batch totals) and reports (n_sys entries, system i's report in reports[i]:
 * its corners, escalated and audit counts, set bits, steps, merges, naive
 * cost and planning time; n_launches is the batch's) may be NULL; when either
 * is given the call synchronizes the stream. */
int pa_batch_execute(pa_batch *batch, pa_bitarray *outs, pa_report *report, pa_report *reports, void *stream);
size_t pa_batch_workspace_bytes(const pa_batch *batch);
/* As pa_plan_op_times, for a batch created with opts->timing == 2: one entry
 * per grouped launch (kind and summed macs of its steps). */
int32_t pa_batch_op_times(pa_batch *batch, double *ms, int32_t *kind, double *macs, int32_t cap);
/* As pa_plan_time_groups, for the batch's merged step table. */
int32_t pa_batch_time_groups(pa_batch *batch, int32_t reps, double *ms, int32_t *kind, double *macs, int32_t cap,
                             void *stream);
/* As pa_plan_set_wait_limit, for the batch's single persistent launch. */
int pa_batch_set_wait_limit(pa_batch *batch, int64_t polls);
void pa_batch_destroy(pa_batch *batch);
/* Solve n_sys independent systems: for each, the solution array on its
 * exposed variables, i.e. the generalized array multiplication of its
 * relation plots over its wiring diagram (Def. "wd", eqn GAM), evaluated as a
 * cluster tree (Sec. 3.5).  pa_batch_create + pa_batch_execute +
 * pa_batch_destroy: outs[i] as for pa_batch_execute (device, caller-owned,
 * dims = system i's exposed resolutions); reports (host, n_sys entries) may
 * be NULL.  Synchronizes the stream.  Errors as for pa_batch_create (failing
 * system named in pa_last_error) and pa_batch_execute. */
int pa_solve_batch(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed, const int32_t *n_exposed,
                   const pa_opts *opts, pa_bitarray *outs, pa_report *reports, void *stream);

/* ---------------------------------------------------------- learned order
 * The tree of pairwise steps only decides the work (Sec. 3.5), and the naive
 * cost r^L of a step (eqn naive_cost) does not say how fast the hardware runs
 * it (matrix cores vs bit streaming, padding, launch latency).  A pa_model is
 * a small MLP (PA_MODEL_FEATURES -> 64 -> 64 -> 1, ReLU, float32) that
 * predicts log2 of a step's duration in microseconds from features of its
 * index groups; PA_ORDER_LEARNED runs a dynamic program over connected sets
 * of relations (all sets if the relation graph is disconnected; greedy above
 * 16 relations) minimizing the sum of predicted step times plus a cost per
 * tree level, with one batched forward pass on the device per 2^18
 * candidate steps; a tree whose naive cost exceeds 4x the exhaustive
 * optimum is replaced by that optimum.  Training data come
 * from the library's own timings (pa_plan_step_samples); forward, backward
 * and the Adam update run in the library's kernels.
 *
 * Parameters are float32 in the flat layout W1[64][F], b1[64], W2[64][64],
 * b2[64], w3[64], b3 (F = PA_MODEL_FEATURES).  A model lives on the device
 * that was current at creation and must be used with that device current
 * (EINVAL otherwise).  Device pointers below are float32 arrays on that
 * device; calls on the same model must not overlap. */
enum { PA_MODEL_FEATURES = 16 };
int32_t pa_model_n_params(void);
int32_t pa_model_n_features(void);
/* New model with uniform He initial weights drawn from SplitMix64(seed), zero
 * biases and zero Adam moments.  EHIP if device memory is unavailable. */
int pa_model_create(uint64_t seed, pa_model **model);
void pa_model_destroy(pa_model *model);
/* Copy the n == pa_model_n_params() parameters to / from host memory;
 * setting them also clears the Adam moments and step count.  EINVAL on a
 * wrong n or a non-finite value. */
int pa_model_get_params(const pa_model *model, float *host_params, int32_t n);
int pa_model_set_params(pa_model *model, const float *host_params, int32_t n);
/* Cost in microseconds that PA_ORDER_LEARNED charges per tree level (the
 * grouped executor launches each level separately); default 6.  EINVAL if
 * negative or not finite. */
int pa_model_set_level_cost(pa_model *model, double us);
/* Y[i] = prediction for features X[i][F], i < n (device pointers; n >= 0). */
int pa_model_forward(pa_model *model, const float *X, int64_t n, float *Y, void *stream);
/* Gradient of the mean squared error (1/n) sum (y_i - T_i)^2 with respect
 * to the parameters, into grad (device, n_params floats; may be NULL), and
 * the loss into *loss (host; may be NULL; then the call synchronizes the
 * stream).  Batch reductions run in a fixed order: results are
 * deterministic.  EINVAL if n < 1. */
int pa_model_gradient(pa_model *model, const float *X, const float *T, int64_t n, float *grad, float *loss,
                      void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on that
 * gradient with learning rate lr > 0; *loss (may be NULL) gets the batch loss
 * before the update. */
int pa_model_train_step(pa_model *model, const float *X, const float *T, int64_t n, float lr, float *loss,
                        void *stream);
/* Checkpoint: one JSON header line, a newline, then the parameters as
 * little-endian float32.  load creates a model on the current device;
 * EINVAL if the file is not a model of this shape. */
int pa_model_save(const pa_model *model, const char *path);
int pa_model_load(const char *path, pa_model **model);
/* Features of the step multiplying the clusters of relation sets s1 and s2
 * (bit r = relation r; disjoint, non-empty) of a system: log2 sizes / 8 of
 * the batch, M, N and shared latent groups, of the scope, output and
 * operands; the path flags (MFMA-eligible, streaming over a shared latent
 * variable, no shared latent variable); scope and output arity / 4; and
 * estimated log2 densities / 8 of both operands and the output: analytic
 * (n generic equations in V unknowns leave a set of dimension V - n; each
 * dimension its projection lacks thins the array by about r/2), or, when the
 * plan measured its plots (opts->measure_density), from the measured plot
 * densities taken as independent: log2 d(S) = min(0, sum of the plots' log2
 * densities + sum of log2 r over the cluster's variables outside its pack).
 * Host-only (analytic densities). */
int pa_step_features(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, uint32_t s1, uint32_t s2,
                     float *features);
/* Training samples from the last execute of a plan created with per_op = 1
 * and timing = 2: for every pairwise step of the tree (in tree order) its
 * features (cap x F floats) and log2 of its measured duration in
 * microseconds (the sum of the step's op launches, from HIP events).  Waits
 * for the events.  Returns the number of steps, or -1 (see pa_last_error). */
int32_t pa_plan_step_samples(pa_plan *plan, float *features, float *log2_us, int32_t cap);

/* ---------------------------------------------------------- autotuning
 * Executor settings for a workload (one system: n_sys = 1), chosen by timing
 * candidates on the device: first the executor (grouped launches, or one
 * persistent launch with 256/512/1024/2048 workgroups), then the plot strip
 * length (1/2/4/8 cells per thread), then the streaming tile (512..32768
 * output bits), then the MFMA K-split target (1, 64, 128, 256, 512, 1024,
 * 2048 work items), then the MFMA operand path (LDS-staged 128x128 or
 * 256x128 tiles, direct, or resident A operands), then (when
 * opts->sparse_pass is 0) the sparse
 * pass alone for every contraction whose B is a plot, then the same with
 * pass pairs fused (sparse_pass 3), each from the best so far.  Every candidate is a batch built
 * with opts (graph capture included if opts->graph), executed once untimed,
 * then reps times between two events on `stream`.  Candidates that exceed
 * the workspace cap are skipped.  best gets the fastest; tried (may be NULL)
 * up to cap of the candidates in order, *n_tried their count.  The result is
 * also cached for opts->autotune.  Allocates outputs and workspaces while
 * tuning; synchronizes the stream. */
typedef struct {
    int32_t single_launch, persist_wg, plot_strip, contract_units, gemm_split, gemm_path;
    int32_t sparse_pass;      /* as in pa_opts: opts->sparse_pass, or 2 or 3 when
                                 that was 0 and the pass alone (3: with fused
                                 pass pairs) was faster                           */
    double ms;                /* milliseconds per execution of the whole workload */
} pa_tuning;
int pa_autotune(const pa_system *systems, int32_t n_sys, const int32_t *const *exposed, const int32_t *n_exposed,
                const pa_opts *opts, int32_t reps, pa_tuning *best, pa_tuning *tried, int32_t cap, int32_t *n_tried,
                void *stream);

/* Solve one system: the solution array A' on the exposed variables (the
 * outer pack), the generalized array multiplication of the relation plots
 * over the system's wiring diagram (Def. "wd", eqn GAM) with every latent
 * variable projected out, evaluated as a cluster tree (Sec. 3.5,
 * Thm "associative": every tree gives the same bits).  pa_plan_create +
 * pa_plan_execute + pa_plan_destroy.  out: device, caller-owned, dims = the
 * exposed resolutions in the listed order; report (host) may be NULL.  The
 * workspace is the library's unless opts->workspace is given (then at least
 * pa_workspace_bytes).  Synchronizes the stream.  Errors as for
 * pa_plan_create and pa_plan_execute. */
int pa_solve_system(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts *opts,
                    pa_bitarray *out, pa_report *report, void *stream);

/* Device bytes of workspace that pa_plan_create / pa_solve_system need for
 * this system and opts (intermediates, tables, executor state: 256-byte
 * aligned), computed by planning on the host without creating a plan or
 * allocating device memory (PA_ORDER_LEARNED runs the model's inference on its
 * device).  opts->autotune, opts->verify_order and opts->measure_density are
 * not applied (the learned order then uses analytic densities): the figure
 * is for the given executor settings and order policy (pass pa_autotune's
 * settings to size an autotuned plan).  Returns 0 on invalid input (EINVAL /
 * ENOMEM cases of pa_plan_create; message in pa_last_error). */
size_t pa_workspace_bytes(const pa_system *sys, const int32_t *exposed, int32_t n_exposed, const pa_opts *opts);

/* Number of set bits of a device bit array (padding is zero by contract). */
int pa_popcount(const pa_bitarray *a, int64_t *count, void *stream);

/* Set bits per tile of a device bit array (its density map): the array's
 * rows (every axis but the last) are cut into blocks of tile_rows rows and
 * its row words into blocks of tile_words words; counts (device, caller-owned,
 * uint32) receives ceil(rows / tile_rows) x ceil(row_words / tile_words)
 * counts, row-major (block of rows outer).  A 0-dim array is one row of one
 * word.  EINVAL: tile sizes < 1, or tile_rows * tile_words * 32 >= 2^32. */
int pa_tile_popcount(const pa_bitarray *a, int32_t tile_rows, int32_t tile_words, uint32_t *counts, void *stream);

/* Measured LDS read rate of the current device, the reference of the
 * LDS-bound fused pass pair's roofline: one workgroup of 1024 threads per CU,
 * every lane reading its own 16-byte slot of a 64 KiB LDS array (free of
 * bank conflicts, 8 independent reads per iteration, 4096 iterations); one
 * warm-up launch, then one launch timed with HIP events on stream.
 * *bytes_per_second (host) receives CUs x 1024 x 4096 x 128 bytes / the
 * timed launch's duration.  Uses the library's small internal workspace
 * (4 KiB per CU).  Returns PA_OK, PA_EINVAL (null output), PA_ENOMEM or
 * PA_EHIP. */
int pa_lds_read_rate(double *bytes_per_second, void *stream);

/* Thread-local message describing the last error. */
const char *pa_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PA_H */
