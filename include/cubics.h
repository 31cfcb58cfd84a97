/*
 * cubics.h - C ABI of the MI355X (gfx950) CSP solver library libcubics.so.
 *
 * The library solves constraint satisfaction problems P = (X, D, C) as the
 * paper states them (Sec. 1.1, "Constraint programming"): X is a set of
 * integer variables, D their finite domains and C a set of constraints, each
 * a subset of the cartesian product of its variables' domains.  A solution
 * assigns every variable a value of its domain so that every constraint
 * holds.  Solving interleaves the three operations of Sec. 1.1 - labeling,
 * constraint propagation and backtracking - and, as Sec. 2.1 prescribes, runs
 * all of them on the GPU after one upload: bitset domains are revised to a
 * fixpoint, and many depth-first subtrees are searched at once by a
 * persistent kernel with per-worker trail stacks and a global work queue.
 *
 * Conventions (all calls):
 *  - Return value 0 (CUBICS_OK) or a negative error code.  On error no handle
 *    is returned, nothing leaks, and cubics_last_error() gives a message
 *    (thread-local, valid until the next call on the same thread).
 *  - Host pointers are read during the call only and copied; the caller may
 *    free them on return.  Device pointers (marked "device") are written on
 *    the context's stream and stay owned by the caller.
 *  - Every call that runs GPU work is synchronous with respect to the host:
 *    it returns after the work finished on the context's stream.
 *  - One context per host thread; contexts are not thread-safe.
 */
#ifndef CUBICS_H
#define CUBICS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ error codes */
#define CUBICS_OK 0
#define CUBICS_EINVAL (-1)       /* malformed argument or instance */
#define CUBICS_ENOMEM (-2)       /* host or device allocation failed */
#define CUBICS_EDEVICE (-3)      /* a HIP call failed */
#define CUBICS_EUNSUPPORTED (-4) /* valid CSP outside the supported range */

/* ------------------------------------------------------- constraint types
 * The flat constraint list given to cubics_load (same layout as the
 * extensional form of Sec. 1.1: a constraint is its scope plus the set of
 * allowed tuples, given either explicitly or by a closed rule).
 *   UNARY      scope (i)    table: ceil(d_i/32) words, bit a <=> value lo_i+a allowed
 *   TABLE2     scope (i,j)  table: d_i rows of ceil(d_j/32) words; bit b of row a
 *                           set <=> the pair (lo_i+a, lo_j+b) is allowed
 *   NEQ        scope (i,j)  params {off}: x_i != x_j + off
 *   LT         scope (i,j)  params {off}: x_i <  x_j + off
 *   QUEENS     scope (i,j)  params {k}:   x_i != x_j and |x_i - x_j| != k
 *   ALLDIFF    scope (v_0..v_{k-1}): pairwise distinct values (domains are
 *              compared in value space; the scope's value span must fit
 *              CUBICS_MAX_DOMAIN); propagated by singleton elimination and a
 *              pigeonhole test
 *   ALLDIFF_GAC  the same constraint, propagated to generalized arc
 *              consistency (a value stays iff some assignment of pairwise
 *              different values uses it: maximum matching and strongly
 *              connected components, the stronger propagation of Sec. 3);
 *              at most 64 variables, else CUBICS_EUNSUPPORTED
 *   LINEAR_LE  scope (v_0..v_{k-1}); params {b, a_0..a_{k-1}}, every a_t > 0:
 *                           sum_t a_t x_{v_t} <= b
 *   LINEAR_LE_AD  the same constraint over distinct variables (a repeated
 *              variable is CUBICS_EINVAL), propagated together with the
 *              ALLDIFF / ALLDIFF_GAC constraints whose variables all lie in
 *              its scope (in constraint order, each sharing no variable with
 *              one taken before; at most 16 of at most 64 variables).  Such
 *              a group's part of the sum is at least its coefficients in
 *              descending order times the smallest values of the union of
 *              its domains in ascending order: the stronger reasoning over
 *              global constraints that Sec. 3 names as a direction.  Same
 *              solutions as LINEAR_LE; fewer or equal surviving values.
 */
enum {
    CUBICS_UNARY = 0,
    CUBICS_TABLE2 = 1,
    CUBICS_NEQ = 2,
    CUBICS_LT = 3,
    CUBICS_QUEENS = 4,
    CUBICS_ALLDIFF = 5,
    CUBICS_LINEAR_LE = 6,
    CUBICS_ALLDIFF_GAC = 7,
    CUBICS_LINEAR_LE_AD = 8
};

/* solve modes */
enum { CUBICS_MODE_FIRST = 0, CUBICS_MODE_ALL = 1, CUBICS_MODE_COUNT = 2 };
/* verdicts */
enum { CUBICS_SAT = 0, CUBICS_UNSAT = 1, CUBICS_LIMIT = 2, CUBICS_CANCELLED = 3 };
/* branching heuristics */
enum { CUBICS_BRANCH_FIRST_FAIL = 0, CUBICS_BRANCH_LEARNED = 1 };
/* revision layouts for binary constraints:
   LANE  one lane per directed propagator, domains in LDS;
   SEG   one lane per value of the revised variable (ballot-assembled), domains in LDS;
   VAR   one lane per variable, domains in registers (instances with at most 64
         variables of at most 32 values, binary constraints only, one constraint
         per variable pair, first-fail, and with 2-way branching only when
         1 + sum_i (d_i - 1) <= 64; other cases fall back to LANE);
   AUTO  the autotuned choice (layout and worker count) for the instance's
         shape, else VAR for a single instance whose tables fit in LDS, else
         SEG for domains wider than 24 values, else LANE. */
enum { CUBICS_LAYOUT_AUTO = 0, CUBICS_LAYOUT_LANE = 1, CUBICS_LAYOUT_SEG = 2, CUBICS_LAYOUT_VAR = 3 };

/* Supported range: 1 <= d_i <= 256 values per variable (at most 8 32-bit
   words per domain); n <= 1024 variables with n * ceil(dmax/32) <= 4096;
   at most 65535 global (ALLDIFF / ALLDIFF_GAC / LINEAR_LE / LINEAR_LE_AD) constraints per
   instance; ALLDIFF_GAC over at most 64 variables. */
#define CUBICS_MAX_DOMAIN 256
#define CUBICS_MAX_VARS 1024

typedef struct cubics_ctx cubics_ctx;
typedef struct cubics_prob cubics_prob;
typedef struct cubics_policy cubics_policy;

typedef struct {
    uint64_t max_nodes;      /* per instance; 0 = unlimited.  Reaching it gives LIMIT */
    uint64_t max_solutions;  /* per instance count cap; 0 = none.  Reaching it gives LIMIT
                                with count == max_solutions */
    int64_t time_ms;         /* wall budget of the search kernel; 0 = none */
    int32_t branching;       /* CUBICS_BRANCH_* */
    int32_t layout;          /* CUBICS_LAYOUT_*; AUTO uses the autotuned choice */
    int64_t split_target;    /* eager subtree splitting until this many subproblems were
                                queued; 0 = no eager split (work is shared by donation) */
    int32_t *sol_buf;        /* device, caller-owned: sol_capacity x n int32 values, or NULL */
    uint64_t sol_capacity;   /* solutions that fit in sol_buf */
    int32_t workers;         /* persistent workers (wavefronts); 0 = fill the device */
    int32_t donate;          /* 1 = busy workers donate subtrees to idle ones (default) */
    const cubics_policy *policy; /* required when branching == LEARNED */
    int32_t tables_in_lds;   /* single-instance solves: 0 = stage the packed constraint
                                tables in LDS once per workgroup when they fit (default),
                                2 = always read them from HBM */
    int32_t explore_pm;      /* trace collection: per-mille of branchings that pick uniformly
                                among the 4 candidates with the smallest domains */
    float *trace_buf;        /* device, caller-owned [trace_capacity][8] floats, or NULL.
                                Each completed subtree under a branching records the
                                branching variable's 5 features, the depth, the instance's
                                index in the batch and the label
                                log2(1 + nodes below the branching).  Subtrees that were
                                split or donated are not recorded. */
    uint64_t trace_capacity;
    uint32_t seed;           /* exploration seed */
    int32_t use_graph;       /* 1 = capture the launch sequence (queue reset + persistent
                                search) in a hipGraph on first use and replay it on later
                                calls with identical launch parameters */
    int32_t two_way;         /* 0 = d-way labeling (one child per value, ascending);
                                1 = 2-way branching: x = a, then x != a, with a the
                                smallest value of the branching variable (the same
                                solutions, another tree: other node counts) */
    int32_t active_per_xcd;  /* batches: k > 0 = one work queue per XCD (8 on MI355X)
                                holding k instances at a time, the next instance admitted
                                to a queue when one of its instances ends, so that the
                                tables an XCD's workers read stay in its L2 (used when
                                B > 8 and the launch has at least 8 workgroups);
                                -1 = every instance queued at launch on one queue;
                                0 = the autotuned choice for the batch's shape (layout
                                AUTO), else one queue */
    const cubics_policy *value_policy; /* NULL = children of a branching in ascending value
                                order; else the learned value order: the children of every
                                d-way branching on x are tried in descending order of
                                this network's score of each value's features (see
                                cubics_value_features), lowest value on ties.  Changes which
                                solution is found first, never the solution set, counts or
                                (all/count mode) node counts.  Domains of at most 64 values,
                                d-way only (EINVAL with two_way or trace recording);
                                runs in the LANE layout */
} cubics_limits;

typedef struct {
    int32_t verdict;     /* CUBICS_SAT / UNSAT / LIMIT / CANCELLED */
    int32_t truncated;   /* 1 if more solutions were found than fit in sol_buf */
    uint64_t count;      /* solutions found (exact unless LIMIT/CANCELLED; then a lower
                            bound, and min(found, max_solutions) under a cap) */
    uint64_t n_written;  /* solutions stored in sol_buf */
    uint64_t nodes;      /* search nodes: the root and every child tried */
    uint64_t fails;      /* nodes whose propagation failed */
    uint64_t revisions;  /* constraint revisions executed (schedule dependent) */
    uint64_t steals;     /* subtrees donated between workers */
    uint64_t alg_bytes;  /* algorithmic domain/table/trail bytes of the revisions and
                            trail operations executed */
    uint64_t tasks;      /* work-queue tasks processed */
    uint64_t traces;     /* trace records written by the launch (see trace_buf) */
    double ms;           /* host wall time of the call */
    double kernel_ms;    /* duration of the search kernel (HIP events on the stream) */
} cubics_result;

/* ---------------------------------------------------------------- errors */

/* Message of the last failed call on this thread ("" if none). */
const char *cubics_last_error(void);

/* --------------------------------------------------------------- context */

/* Create a context on HIP device `device`, issuing work on `hip_stream`
   (a hipStream_t; NULL = the null stream).  The context owns scratch device
   memory (work queue, trail stacks) that grows on demand. */
int cubics_create(int32_t device, void *hip_stream, cubics_ctx **out);
void cubics_destroy(cubics_ctx *ctx);
int cubics_set_stream(cubics_ctx *ctx, void *hip_stream);
/* Ask a running solve on this context to stop (safe from another thread);
   the solve then returns verdict CANCELLED.  cubics_solve clears the flag on entry. */
void cubics_cancel(cubics_ctx *ctx);

/* ------------------------------------------------------------------ load */

/* Pack one CSP (Sec. 2.1: the host builds the data structures and moves
   them to GPU memory once).  Arrays (host):
     lo[n], dsize[n]                 value range of each variable
     init_bits[n * W] or NULL        W = ceil(max dsize / 32); optional initial domains
                                     (bit a of row i = value lo_i + a); an empty initial
                                     domain is not an error (the solve returns UNSAT)
     type[m], arity[m]               CUBICS_* type and scope size of each constraint
     var_off[m+1], vars[]            scope of constraint c = vars[var_off[c] .. var_off[c+1])
     par_off[m+1], params[]          integer parameters (see the type list)
     tab_off[m+1], tabs[]            packed bit rows (UNARY, TABLE2), in uint32 words
   Errors: EINVAL for a variable index out of range, a wrong arity, repeated
   scope variables, dsize < 1, a table of the wrong length, a non-positive
   linear coefficient; EUNSUPPORTED for dsize > 256, n > 1024, an ALLDIFF
   over variables with different lo, or a linear sum that may overflow int64.
   n == 0 is valid (one empty solution). */
int cubics_load(cubics_ctx *ctx, int32_t n, const int32_t *lo, const int32_t *dsize,
                const uint32_t *init_bits, int32_t m, const int32_t *type,
                const int32_t *arity, const int64_t *var_off, const int32_t *vars,
                const int64_t *par_off, const int64_t *params, const int64_t *tab_off,
                const uint32_t *tabs, cubics_prob **out);
void cubics_free(cubics_prob *prob);
/* n, W (words per domain) and the number of propagators of a loaded problem. */
int cubics_prob_info(const cubics_prob *prob, int32_t *n, int32_t *W, int32_t *n_units,
                     int32_t *n_global);

/* ------------------------------------------------------------- propagate */

/* Root propagation only (Sec. 1.1 "constraint propagation"): the initial
   domains restricted by UNARY constraints, revised on the GPU to the fixpoint
   of all constraints.  out_bits (host, n * W words) receives the fixpoint
   domains; *failed = 1 if a domain emptied or a constraint test failed. */
int cubics_root(cubics_prob *prob, int32_t layout, uint32_t *out_bits, int32_t *failed);

/* ----------------------------------------------------------------- solve */

/* Search one problem (Sec. 1.1 labeling + propagation + backtracking, Sec. 2.2
   parallel propagation and per-domain save/restore), entirely on the GPU.
   mode FIRST: stop at the first solution and store it in sol_buf[0..n);
   ALL: count every solution and store up to sol_capacity of them (unordered);
   COUNT: count only (sol_buf may still receive up to sol_capacity).
   Branching: first-fail (fewest values, lowest index on ties), values in
   ascending order; LEARNED picks the variable by the policy network instead,
   which changes the order of the search but never its result.
   Hitting max_nodes / max_solutions / time_ms is a verdict (LIMIT), not an
   error.  Workers check them periodically: max_nodes every 128 nodes of a
   worker, so a search may run up to 128 nodes per worker past it; a stop
   (time_ms, cancel, another worker's find-first solution) is seen within
   2048 nodes of a worker (the register layout without a node budget polls
   that rarely: more frequent polls split its searches' tails too finely).
   `limits` may be NULL (no limits, defaults). */
int cubics_solve(cubics_prob *prob, int32_t mode, const cubics_limits *limits,
                 cubics_result *result);

/* Solve B problems in one persistent launch (work-queue tasks are tagged by
   instance).  limits[b] gives the per-instance max_nodes, max_solutions,
   sol_buf and sol_capacity; the launch-wide knobs (time_ms, branching,
   layout, split_target, workers, donate, policy) come from limits[0].
   results[b] receives each instance's verdict and counters; kernel_ms and ms
   are those of the whole launch.  All problems must come from contexts on the
   same device; the work runs on the first problem's context stream. */
int cubics_solve_batch(cubics_prob *const *probs, int32_t B, int32_t mode,
                       const cubics_limits *limits, cubics_result *results);

/* Allocation-free variant of cubics_solve_batch, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc).  Same arguments, semantics and
   results as cubics_solve_batch, except that every device buffer of the
   launch (instance descriptors, per-instance counters, the work queue, the
   workers' trail stacks) comes from a static device array of
   CUBICS_STATIC_SCRATCH_MIB MiB that each GPU holds from its first use until
   the process ends; the call allocates no device memory itself (the
   problems, the context and the caller's solution buffers exist already).
   The worker count shrinks until the trails fit the array, so a launch may
   run on fewer workers than cubics_solve_batch would use.  Errors: as
   cubics_solve_batch, plus EUNSUPPORTED when even one worker does not fit
   (B descriptors + queue + one trail exceed the array) and EINVAL for
   use_graph or trace recording, which need allocations.  Every call on one
   GPU shares that GPU's array and the last call's contents stay in it:
   calls that overlap on one GPU (other threads, other streams) race and
   must be serialised by the caller. */
#define CUBICS_STATIC_SCRATCH_MIB 256
int cubics_solve_batch_static(cubics_prob *const *probs, int32_t B, int32_t mode,
                              const cubics_limits *limits, cubics_result *results);

/* Autotuner: run these problems for time_ms of search under each revision
   layout they admit (LANE, SEG, VAR) and each of CUBICS_AUTOTUNE_DIVS worker
   counts (the occupancy-limited maximum divided by 1, 2 and 4: a small
   search tree finishes sooner on fewer workers, whose idle polls and task
   hand-offs cost less), measure search nodes per ms, and remember the fastest
   pair (a smaller worker count of the same layout must be 5% faster to win)
   for the first problem's shape bucket (domain words, domain size,
   variable count, constraint kinds).  For a batch (B > 8) it then tries one
   queue per XCD with 4, 8, 16 and 32 instances active on each (see
   active_per_xcd), kept if 5% faster than one queue.  Later solves with
   layout AUTO, workers 0 and active_per_xcd 0 on the same context use the
   choice.  *chosen, *chosen_div and *chosen_active (nullable) receive the
   layout, the divisor and the instances per XCD (0 = one queue); rates
   (nullable, host, 3 * CUBICS_AUTOTUNE_DIVS doubles) receives the measured
   nodes per ms at [(layout - 1) * CUBICS_AUTOTUNE_DIVS + divisor index]
   (one queue), 0 where a layout is not admitted.  The runs use limits[]
   (NULL: none) with time_ms added. */
enum { CUBICS_AUTOTUNE_DIVS = 3 };
int cubics_autotune(cubics_prob *const *probs, int32_t B, int32_t mode, const cubics_limits *limits,
                    int64_t time_ms, int32_t *chosen, int32_t *chosen_div, int32_t *chosen_active,
                    double *rates);

/* ------------------------------------------- large-neighbourhood search
 * Minimise sum_i obj[i] * x_i (every obj[i] >= 0, at least one > 0) over the
 * solutions of the CSP given as for cubics_load (the parallel large-
 * neighbourhood search the paper names as future work, Sec. 3).  Round 0
 * finds a first solution; each later round adds sum obj[i] x_i <= best - 1
 * and solves `neighborhoods` copies in one persistent launch (find-first,
 * max_nodes each): copy 0 frees every variable - if it is UNSAT the
 * incumbent is optimal and the search stops - and the others fix each
 * variable to its incumbent value except a random relax_pm per mille.  The
 * best solution found is written to best (host, n int32 values).  Stops
 * after `rounds` rounds (0 = until optimal or time_ms), when time_ms (0 =
 * none) has passed, or on proof. */
typedef struct {
    int32_t neighborhoods;   /* copies per round, 1..65536 */
    int32_t rounds;          /* 0 = no round limit */
    int32_t relax_pm;        /* per mille of variables freed in copies 1.., 1..1000 */
    uint32_t seed;           /* neighbourhood choice */
    uint64_t max_nodes;      /* node budget of each copy; 0 = none */
    int64_t time_ms;         /* overall wall budget; 0 = none */
} cubics_lns_params;

typedef struct {
    int64_t objective;       /* of the best solution found (valid if found) */
    int32_t found;           /* 1 if any solution was found */
    int32_t optimal;         /* 1 if copy 0 proved that nothing better exists */
    int32_t rounds;          /* rounds run */
    int32_t improvements;    /* rounds that improved the incumbent (after round 0) */
    uint64_t nodes;          /* search nodes over all copies and rounds */
    double ms;               /* host wall time of the call */
} cubics_lns_result;

int cubics_lns(cubics_ctx *ctx, int32_t n, const int32_t *lo, const int32_t *dsize,
               const uint32_t *init_bits, int32_t m, const int32_t *type, const int32_t *arity,
               const int64_t *var_off, const int32_t *vars, const int64_t *par_off,
               const int64_t *params, const int64_t *tab_off, const uint32_t *tabs,
               const int64_t *obj, const cubics_lns_params *lp, int32_t *best,
               cubics_lns_result *res);

/* -------------------------------------------------------- learned policy
 * The branching network (variable ordering, used when branching == LEARNED):
 * features f (5 per candidate variable) -> 64 ReLU units -> 1 output, the
 * predicted log2(1 + size of the subtree below branching on the variable);
 * the candidate with the smallest prediction is branched on (lowest index on
 * ties).  theta (449 floats, host) = W1[64][5] (row = hidden unit), b1[64],
 * w2[64], b2.  Weights are used in bf16 (round to nearest even) with fp32
 * accumulation on the matrix cores; theta stays the fp32 master copy.  The
 * policy never changes what propagation computes, only the search order. */

/* The 5 policy features of every variable at a search node whose domains are
   dom_bits (host, n * W words as cubics_root returns them; NULL = the
   problem's initial domains) at the given depth (number of branchings above
   it, >= 0), with no failures counted: |D_i| / d_i, static degree / (n - 1),
   mean static tightness of the variable's constraints, depth / n,
   log2(1 + failures) = 0.  out (host, n * 5 floats) receives them, row i =
   variable i.  The values are those the branching step computes. */
int cubics_features(cubics_prob *prob, const uint32_t *dom_bits, int32_t depth, float *out);

/* The 5 value features of every value a < 32 W of variable x at a search
   node whose domains are dom_bits (host, n * W words; NULL = the initial
   domains) at the given depth: out (host, 32 W * 5 floats), row a =
   a / d_x, the mean and the smallest, over x's table constraints, of the
   fraction of the other variable's current values that x = lo_x + a
   supports (1 when x has no table constraint), depth / n, |D_x| / d_x;
   zeros for values not in D_x.  The values the learned value order
   computes.  EUNSUPPORTED for domains wider than 64 values. */
int cubics_value_features(cubics_prob *prob, const uint32_t *dom_bits, int32_t depth, int32_t x, float *out);

/* Upload theta (copied) and zero the optimizer state. */
int cubics_policy_create(cubics_ctx *ctx, const float *theta, cubics_policy **out);
void cubics_policy_free(cubics_policy *policy);
int cubics_policy_get(const cubics_policy *policy, float *theta);
int cubics_policy_set(cubics_policy *policy, const float *theta);
/* y_dev[s] = network output for row s of x_dev (device, fp32 rows of stride
   ld >= 5 floats, features in columns 0..4 - trace records have ld = 8).
   Inputs are rounded to bf16 as in the search kernel. */
int cubics_mlp_forward(const cubics_policy *policy, const float *x_dev, int32_t ld, int64_t N, float *y_dev);
/* Gradient of the mean squared error mean_s (y_s - t_s)^2 with respect to
   theta (targets t_dev[s * ldt], device), written to grad_dev (device, 449
   floats; NULL = internal) and the loss to loss_dev (device, 1 float; NULL =
   internal).  The bf16 rounding of weights, inputs and activations counts as
   the identity (straight-through). */
int cubics_mlp_grad(const cubics_policy *policy, const float *x_dev, int32_t ld, const float *t_dev,
                    int32_t ldt, int64_t N, float *grad_dev, float *loss_dev);
/* One full-batch training step: gradient, Adam (beta1 0.9, beta2 0.999,
   eps 1e-8, bias-corrected, step >= 1) on theta, re-rounding of the bf16
   weights.  *loss_host (nullable) receives the loss before the step. */
int cubics_mlp_train_step(cubics_policy *policy, const float *x_dev, int32_t ld, const float *t_dev,
                          int32_t ldt, int64_t N, float lr, int32_t step, float *loss_host);

#ifdef __cplusplus
}
#endif

#endif /* CUBICS_H */
