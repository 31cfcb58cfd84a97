/*
 * CPU ORACLE - TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded reference for what the solver computes,
 * written from the paper's problem statement (Sec. 1.1): a CSP is
 * P = (X, D, C); a constraint is a subset of the cartesian product of its
 * variables' domains; a solution assigns every variable a value of its domain
 * so that all constraints hold.  The solver is built from the three
 * operations the paper lists in Sec. 1.1: labeling (assign a variable one
 * value of its domain), constraint propagation (remove values that cannot
 * occur in any solution) and backtracking (restore the domains at a dead end,
 * record the solution on success).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * this file.  It shares no code, header or table with the GPU library.
 *
 * Readings of what the paper leaves open (each applies to the GPU solver too):
 *  - labeling assigns one value at a time, values in ascending order
 *    (d-way branching); the variable is the one with the fewest values among
 *    those with two or more, lowest index on ties (first-fail);
 *  - propagation reaches the fixpoint of: arc consistency on every binary
 *    constraint (table, !=, <, queens pair as one constraint), singleton
 *    elimination plus a pigeonhole test for all-different, and bounds
 *    reasoning for sum a_t x_t <= b with positive a_t; unary constraints
 *    restrict the root domains; the all-different of type 7 is propagated
 *    to generalized arc consistency instead (the stronger propagation the
 *    paper names as future work, Sec. 3), and the linear <= of type 8 is
 *    bounded together with the all-different constraints inside its scope
 *    (revise_linear_ad);
 *  - a node is every propagation call: the root and every child tried,
 *    failed children included;
 *  - a table constraint is given over the original domains and is
 *    intersected with the current domains when revised.
 *
 * Domains here are byte arrays (one byte per value), not bit sets.
 *
 * Parity status: every function in this file is pinned by the CPU tests
 * (brute force, the paper's worked example, n-queens counts, closed forms,
 * tree-CSP counts, definition-level searches); none is "parity unpinned".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { T_UNARY = 0, T_TABLE2 = 1, T_NEQ = 2, T_LT = 3, T_QUEENS = 4, T_ALLDIFF = 5, T_LINEAR = 6,
       T_ALLDIFF_GAC = 7, T_LINEAR_AD = 8 };
enum { AD_GROUPS_MAX = 16 };
enum { M_FIRST = 0, M_ALL = 1, M_COUNT = 2 };
enum { V_SAT = 0, V_UNSAT = 1, V_LIMIT = 2 };

typedef struct {
    int32_t n, m;
    const int32_t *lo, *dsize;
    const uint32_t *init;      /* nullable, n x W words, W = ceil(dmax/32) */
    const int32_t *type, *arity;
    const int64_t *var_off;
    const int32_t *vars;
    const int64_t *par_off;
    const int64_t *params;
    const int64_t *tab_off;
    const uint32_t *tabs;
} orc_problem;

typedef struct {
    int32_t verdict;
    int32_t truncated;
    int64_t count, n_written, nodes, fails, revisions, max_depth;
} orc_stats;

/* one propagator: a binary arc (revise one scope var against the other) or a
   whole global constraint */
typedef struct {
    int con;
    int dir;   /* binary: 0 revises scope[0] against scope[1], 1 the reverse */
} prop_t;

typedef struct {
    const orc_problem *P;
    int n, dmax, W;
    int nprop;
    prop_t *prop;
    int *watch_off, *watch;   /* var -> propagators whose scope contains it */
    /* AC-3 queue */
    int *queue, qhead, qtail, qcap;
    unsigned char *inq;
    /* search */
    int mode;
    int two_way;  /* 1: children x = min D_x, then x != min D_x */
    int64_t max_nodes, cap;
    int32_t *sols;
    int64_t sol_cap;
    int stop;
    orc_stats st;
} ctx_t;

/* ---------------------------------------------------------------- helpers */

static int64_t value_of(const ctx_t *C, int i, int a) { return (int64_t)C->P->lo[i] + a; }

static int dom_size(const ctx_t *C, const unsigned char *D, int i) {
    int s = 0;
    for (int a = 0; a < C->P->dsize[i]; ++a) s += D[(int64_t)i * C->dmax + a];
    return s;
}

static int dom_min(const ctx_t *C, const unsigned char *D, int i) {
    for (int a = 0; a < C->P->dsize[i]; ++a)
        if (D[(int64_t)i * C->dmax + a]) return a;
    return -1;
}

static int tab_bit(const ctx_t *C, int c, int a, int b) {
    /* TABLE2 row a (first scope var) has ceil(d_j/32) words */
    const orc_problem *P = C->P;
    int j = P->vars[P->var_off[c] + 1];
    int Wj = (P->dsize[j] + 31) / 32;
    const uint32_t *t = P->tabs + P->tab_off[c];
    return (t[(int64_t)a * Wj + b / 32] >> (b % 32)) & 1u;
}

/* Is the pair (value vi of scope[0], value vj of scope[1]) allowed by binary
   constraint c?  ai/bj are the value indices (for the table form). */
static int pair_allowed(const ctx_t *C, int c, int ai, int bj) {
    const orc_problem *P = C->P;
    int i = P->vars[P->var_off[c]], j = P->vars[P->var_off[c] + 1];
    int64_t vi = value_of(C, i, ai), vj = value_of(C, j, bj);
    const int64_t *par = P->params + P->par_off[c];
    switch (P->type[c]) {
    case T_TABLE2: return tab_bit(C, c, ai, bj);
    case T_NEQ: return vi != vj + par[0];
    case T_LT: return vi < vj + par[0];
    case T_QUEENS: {
        int64_t diff = vi - vj;
        if (diff < 0) diff = -diff;
        return vi != vj && diff != par[0];
    }
    default: return 0;
    }
}

/* ------------------------------------------------------------- revisions */

/* Arc consistency for one direction: keep a value of the revised variable iff
   some value of the other variable forms an allowed pair with it.  Returns
   bitmask of changed (1) / emptied (2). */
static int revise_binary(ctx_t *C, unsigned char *D, int c, int dir, int *changed_var) {
    const orc_problem *P = C->P;
    int s0 = P->vars[P->var_off[c]], s1 = P->vars[P->var_off[c] + 1];
    int x = dir == 0 ? s0 : s1;   /* revised */
    int y = dir == 0 ? s1 : s0;   /* support side */
    unsigned char *Dx = D + (int64_t)x * C->dmax, *Dy = D + (int64_t)y * C->dmax;
    int changed = 0, left = 0;
    for (int a = 0; a < P->dsize[x]; ++a) {
        if (!Dx[a]) continue;
        int supported = 0;
        for (int b = 0; b < P->dsize[y] && !supported; ++b) {
            if (!Dy[b]) continue;
            supported = dir == 0 ? pair_allowed(C, c, a, b) : pair_allowed(C, c, b, a);
        }
        if (!supported) { Dx[a] = 0; changed = 1; } else ++left;
    }
    *changed_var = x;
    return changed | (left == 0 ? 2 : 0);
}

/* All-different: every variable whose domain is a single value w removes w
   from every other scope variable (two equal singletons empty each other);
   then fail if the union of the scope domains has fewer values than the
   scope has variables (pigeonhole). */
static int revise_alldiff(ctx_t *C, unsigned char *D, int c, unsigned char *chg) {
    const orc_problem *P = C->P;
    int k = P->arity[c];
    const int32_t *sc = P->vars + P->var_off[c];
    int64_t *sval = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    int *issing = (int *)malloc(sizeof(int) * (size_t)k);
    for (int t = 0; t < k; ++t) {
        issing[t] = dom_size(C, D, sc[t]) == 1;
        sval[t] = issing[t] ? value_of(C, sc[t], dom_min(C, D, sc[t])) : 0;
    }
    int status = 0;
    for (int t = 0; t < k; ++t) {
        if (!issing[t]) continue;
        for (int u = 0; u < k; ++u) {
            if (u == t) continue;
            int x = sc[u];
            int64_t a = sval[t] - P->lo[x];
            if (a >= 0 && a < P->dsize[x] && D[(int64_t)x * C->dmax + a]) {
                D[(int64_t)x * C->dmax + a] = 0;
                chg[x] = 1;
                status |= 1;
            }
        }
    }
    for (int u = 0; u < k; ++u)
        if (dom_size(C, D, sc[u]) == 0) status |= 2;
    if (!(status & 2)) {
        /* pigeonhole over the values of the scope */
        int64_t vmin = INT64_MAX, vmax = INT64_MIN;
        for (int u = 0; u < k; ++u) {
            int x = sc[u];
            if (P->lo[x] < vmin) vmin = P->lo[x];
            if ((int64_t)P->lo[x] + P->dsize[x] - 1 > vmax) vmax = (int64_t)P->lo[x] + P->dsize[x] - 1;
        }
        int64_t span = vmax - vmin + 1;
        unsigned char *seen = (unsigned char *)calloc((size_t)span, 1);
        int64_t distinct = 0;
        for (int u = 0; u < k; ++u) {
            int x = sc[u];
            for (int a = 0; a < P->dsize[x]; ++a)
                if (D[(int64_t)x * C->dmax + a]) {
                    int64_t v = value_of(C, x, a) - vmin;
                    if (!seen[v]) { seen[v] = 1; ++distinct; }
                }
        }
        free(seen);
        if (distinct < k) status |= 2;
    }
    free(sval);
    free(issing);
    return status;
}

/* Kuhn's augmenting path from scope variable u (index into the scope) over
   the value indices of its domain; mv[v] = scope index matched to value v. */
static int kuhn_try(const unsigned char *adj, int span, int u, int *mv, unsigned char *seen) {
    for (int v = 0; v < span; ++v) {
        if (!adj[(int64_t)u * span + v] || seen[v]) continue;
        seen[v] = 1;
        if (mv[v] < 0 || kuhn_try(adj, span, mv[v], mv, seen)) {
            mv[v] = u;
            return 1;
        }
    }
    return 0;
}

/* Does the scope have an assignment of pairwise different values from adj
   (scope index x value index)?  A maximum bipartite matching covers the scope. */
static int has_sdr(const unsigned char *adj, int k, int span, int *mv, unsigned char *seen) {
    for (int v = 0; v < span; ++v) mv[v] = -1;
    for (int u = 0; u < k; ++u) {
        memset(seen, 0, (size_t)span);
        if (!kuhn_try(adj, span, u, mv, seen)) return 0;
    }
    return 1;
}

/* All-different to generalized arc consistency, from the definition: value v
   stays in D_x iff the scope can take pairwise different values from its
   domains with x = v (one matching test per variable-value pair). */
static int revise_alldiff_gac(ctx_t *C, unsigned char *D, int c, unsigned char *chg) {
    const orc_problem *P = C->P;
    int k = P->arity[c];
    const int32_t *sc = P->vars + P->var_off[c];
    int64_t vmin = INT64_MAX, vmax = INT64_MIN;
    for (int u = 0; u < k; ++u) {
        int x = sc[u];
        if (P->lo[x] < vmin) vmin = P->lo[x];
        if ((int64_t)P->lo[x] + P->dsize[x] - 1 > vmax) vmax = (int64_t)P->lo[x] + P->dsize[x] - 1;
    }
    int span = (int)(vmax - vmin + 1);
    unsigned char *adj = (unsigned char *)calloc((size_t)k * span, 1);
    unsigned char *keep = (unsigned char *)calloc((size_t)k * span, 1);
    unsigned char *seen = (unsigned char *)malloc((size_t)span);
    int *mv = (int *)malloc(sizeof(int) * (size_t)span);
    for (int u = 0; u < k; ++u) {
        int x = sc[u];
        for (int a = 0; a < P->dsize[x]; ++a)
            if (D[(int64_t)x * C->dmax + a]) adj[(int64_t)u * span + (value_of(C, x, a) - vmin)] = 1;
    }
    for (int u = 0; u < k; ++u) {
        unsigned char *row = (unsigned char *)malloc((size_t)span);
        memcpy(row, adj + (int64_t)u * span, (size_t)span);
        for (int v = 0; v < span; ++v) {
            if (!row[v]) continue;
            memset(adj + (int64_t)u * span, 0, (size_t)span);
            adj[(int64_t)u * span + v] = 1;
            keep[(int64_t)u * span + v] = (unsigned char)has_sdr(adj, k, span, mv, seen);
        }
        memcpy(adj + (int64_t)u * span, row, (size_t)span);
        free(row);
    }
    int status = 0;
    for (int u = 0; u < k; ++u) {
        int x = sc[u];
        for (int a = 0; a < P->dsize[x]; ++a) {
            unsigned char *cell = D + (int64_t)x * C->dmax + a;
            if (*cell && !keep[(int64_t)u * span + (value_of(C, x, a) - vmin)]) {
                *cell = 0;
                chg[x] = 1;
                status |= 1;
            }
        }
        if (dom_size(C, D, x) == 0) status |= 2;
    }
    free(adj); free(keep); free(seen); free(mv);
    return status;
}

/* sum_t a_t x_t <= b with every a_t > 0: with S the sum of a_t * min(D_t),
   fail if S > b; otherwise remove every value v of D_t with
   a_t * v + (S - a_t * min(D_t)) > b. */
static int revise_linear(ctx_t *C, unsigned char *D, int c, unsigned char *chg) {
    const orc_problem *P = C->P;
    int k = P->arity[c];
    const int32_t *sc = P->vars + P->var_off[c];
    const int64_t *par = P->params + P->par_off[c];
    int64_t b = par[0];
    int64_t S = 0;
    for (int t = 0; t < k; ++t) {
        int mn = dom_min(C, D, sc[t]);
        if (mn < 0) return 2;
        S += par[1 + t] * value_of(C, sc[t], mn);
    }
    if (S > b) return 2;
    int status = 0;
    for (int t = 0; t < k; ++t) {
        int x = sc[t];
        int64_t at = par[1 + t];
        int64_t rest = S - at * value_of(C, x, dom_min(C, D, x));
        for (int a = 0; a < P->dsize[x]; ++a) {
            unsigned char *cell = D + (int64_t)x * C->dmax + a;
            if (*cell && at * value_of(C, x, a) + rest > b) { *cell = 0; chg[x] = 1; status |= 1; }
        }
    }
    return status;
}

/* sum_t a_t x_t <= b (every a_t > 0) propagated together with the
   all-different constraints (types 5 and 7) whose scopes lie inside its
   scope: in constraint order, each one that shares no variable with a group
   taken before becomes a group (at most AD_GROUPS_MAX).  The variables of a
   group take pairwise different values, so the group's part of the sum is
   at least L_g = sum_j a_(j) u_j, with the group's coefficients sorted in
   descending order and u_1 < u_2 < ... the smallest values of the union of
   its domains (the largest coefficient meets the smallest value).  The
   lower bound of the whole sum is
       S = sum over ungrouped t of a_t min D_t + sum over groups of max(P_g, L_g),
   P_g the group's sum of a_t min D_t.  Fail if S > b, or if a group's union
   holds fewer values than the group has variables.  Remove a value v of x_t
   when a_t v + rest_t > b, with rest_t = S - a_t min D_t for ungrouped t and
   S - (max(P_g, L_g) - P_g) - a_t min D_t for t in group g: the other
   variables of the group contribute at least P_g - a_t min D_t.  Every
   quantity only grows as domains shrink, so the propagator is monotone. */
static int ad_groups(const ctx_t *C, int c, int *grp /* [k]: group of each scope position or -1 */) {
    const orc_problem *P = C->P;
    int k = P->arity[c];
    const int32_t *sc = P->vars + P->var_off[c];
    for (int t = 0; t < k; ++t) grp[t] = -1;
    int G = 0;
    for (int c2 = 0; c2 < P->m && G < AD_GROUPS_MAX; ++c2) {
        if (P->type[c2] != T_ALLDIFF && P->type[c2] != T_ALLDIFF_GAC) continue;
        int k2 = P->arity[c2];
        const int32_t *s2 = P->vars + P->var_off[c2];
        int pos[64], ok = k2 <= 64;
        for (int u = 0; u < k2 && ok; ++u) {
            pos[u] = -1;
            for (int t = 0; t < k; ++t)
                if (sc[t] == s2[u]) pos[u] = t;
            ok = pos[u] >= 0 && grp[pos[u]] < 0;
        }
        if (!ok) continue;
        for (int u = 0; u < k2; ++u) grp[pos[u]] = G;
        G++;
    }
    return G;
}

static int cmp_i64_desc(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return a < b ? 1 : (a > b ? -1 : 0);
}
static int cmp_i64_asc(const void *x, const void *y) { return -cmp_i64_desc(x, y); }

static int revise_linear_ad(ctx_t *C, unsigned char *D, int c, unsigned char *chg) {
    const orc_problem *P = C->P;
    int k = P->arity[c];
    const int32_t *sc = P->vars + P->var_off[c];
    const int64_t *par = P->params + P->par_off[c];
    int64_t b = par[0];
    int *grp = (int *)malloc(sizeof(int) * (size_t)k);
    int64_t *vals = (int64_t *)malloc(sizeof(int64_t) * (size_t)64 * (size_t)C->dmax);
    int G = ad_groups(C, c, grp);
    int64_t S = 0, delta[AD_GROUPS_MAX];
    int status = 0;
    for (int t = 0; t < k; ++t) {
        if (dom_min(C, D, sc[t]) < 0) { status = 2; goto done; }
        if (grp[t] < 0) S += par[1 + t] * value_of(C, sc[t], dom_min(C, D, sc[t]));
    }
    for (int g = 0; g < G; ++g) {
        int64_t Pg = 0, coef[64];
        int kg = 0, nv = 0;
        for (int t = 0; t < k; ++t) {
            if (grp[t] != g) continue;
            int x = sc[t];
            Pg += par[1 + t] * value_of(C, x, dom_min(C, D, x));
            coef[kg++] = par[1 + t];
            for (int a = 0; a < P->dsize[x]; ++a)
                if (D[(int64_t)x * C->dmax + a]) vals[nv++] = value_of(C, x, a);
        }
        qsort(vals, (size_t)nv, sizeof(int64_t), cmp_i64_asc);
        int nu = 0;  /* distinct values, in place */
        for (int q = 0; q < nv; ++q)
            if (nu == 0 || vals[q] != vals[nu - 1]) vals[nu++] = vals[q];
        if (nu < kg) { status = 2; goto done; }
        qsort(coef, (size_t)kg, sizeof(int64_t), cmp_i64_desc);
        int64_t Lg = 0;
        for (int j = 0; j < kg; ++j) Lg += coef[j] * vals[j];
        int64_t mx = Lg > Pg ? Lg : Pg;
        S += mx;
        delta[g] = mx - Pg;
    }
    if (S > b) { status = 2; goto done; }
    for (int t = 0; t < k; ++t) {
        int x = sc[t];
        int64_t at = par[1 + t];
        int64_t rest = S - at * value_of(C, x, dom_min(C, D, x)) - (grp[t] >= 0 ? delta[grp[t]] : 0);
        for (int a = 0; a < P->dsize[x]; ++a) {
            unsigned char *cell = D + (int64_t)x * C->dmax + a;
            if (*cell && at * value_of(C, x, a) + rest > b) { *cell = 0; chg[x] = 1; status |= 1; }
        }
    }
done:
    free(vals);
    free(grp);
    return status;
}

/* ----------------------------------------------------------- propagation */

static void enqueue(ctx_t *C, int p) {
    if (C->inq[p]) return;
    C->inq[p] = 1;
    C->queue[C->qtail] = p;
    C->qtail = (C->qtail + 1) % C->qcap;
}

static void enqueue_var(ctx_t *C, int v) {
    for (int t = C->watch_off[v]; t < C->watch_off[v + 1]; ++t) enqueue(C, C->watch[t]);
}

/* AC-3 style: pop a propagator, revise, and on every domain change put back
   every propagator whose scope contains the changed variable.  Returns 0 at
   the fixpoint, 1 on failure (an empty domain or a failed test). */
static int propagate(ctx_t *C, unsigned char *D, unsigned char *chg) {
    while (C->qhead != C->qtail) {
        int p = C->queue[C->qhead];
        C->qhead = (C->qhead + 1) % C->qcap;
        C->inq[p] = 0;
        C->st.revisions++;
        int c = C->prop[p].con, ty = C->P->type[c];
        int status;
        if (ty == T_ALLDIFF || ty == T_LINEAR || ty == T_ALLDIFF_GAC || ty == T_LINEAR_AD) {
            memset(chg, 0, (size_t)C->n);
            status = ty == T_ALLDIFF     ? revise_alldiff(C, D, c, chg)
                     : ty == T_LINEAR    ? revise_linear(C, D, c, chg)
                     : ty == T_LINEAR_AD ? revise_linear_ad(C, D, c, chg)
                                         : revise_alldiff_gac(C, D, c, chg);
            if (status & 2) goto fail;
            for (int v = 0; v < C->n; ++v)
                if (chg[v]) enqueue_var(C, v);
        } else {
            int x;
            status = revise_binary(C, D, c, C->prop[p].dir, &x);
            if (status & 2) goto fail;
            if (status & 1) enqueue_var(C, x);
        }
    }
    return 0;
fail:
    while (C->qhead != C->qtail) {
        C->inq[C->queue[C->qhead]] = 0;
        C->qhead = (C->qhead + 1) % C->qcap;
    }
    return 1;
}

/* --------------------------------------------------------------- search */

static int solution_test(const ctx_t *C, const unsigned char *D) {
    for (int i = 0; i < C->n; ++i)
        if (dom_size(C, D, i) != 1) return 0;
    return 1;
}

static void record(ctx_t *C, const unsigned char *D) {
    if (C->sols && C->st.n_written < C->sol_cap) {
        int32_t *row = C->sols + C->st.n_written * C->n;
        for (int i = 0; i < C->n; ++i) row[i] = (int32_t)value_of(C, i, dom_min(C, D, i));
        C->st.n_written++;
    } else if (C->sols && C->mode != M_COUNT) {
        C->st.truncated = 1;
    }
    C->st.count++;
    if (C->mode == M_FIRST) C->stop = 1;
    if (C->cap > 0 && C->st.count >= C->cap) C->stop = 2;
}

static int choose_var(const ctx_t *C, const unsigned char *D) {
    int best = -1, bsize = 0;
    for (int i = 0; i < C->n; ++i) {
        int s = dom_size(C, D, i);
        if (s >= 2 && (best < 0 || s < bsize)) { best = i; bsize = s; }
    }
    return best;
}

/* D is a propagated, non-failed node */
static void dfs(ctx_t *C, unsigned char *D, int depth, unsigned char *chg) {
    if (depth > C->st.max_depth) C->st.max_depth = depth;
    if (solution_test(C, D)) { record(C, D); return; }
    int x = choose_var(C, D);
    size_t bytes = (size_t)C->n * (size_t)C->dmax;
    unsigned char *child = (unsigned char *)malloc(bytes);
    if (C->two_way) {
        /* 2-way branching: x = a with a the smallest value, then x != a */
        int a = dom_min(C, D, x);
        for (int side = 0; side < 2 && !C->stop; ++side) {
            if (C->max_nodes > 0 && C->st.nodes >= C->max_nodes) { C->stop = 3; break; }
            memcpy(child, D, bytes);
            if (side == 0) {
                memset(child + (int64_t)x * C->dmax, 0, (size_t)C->dmax);
                child[(int64_t)x * C->dmax + a] = 1;
            } else {
                child[(int64_t)x * C->dmax + a] = 0;
            }
            C->st.nodes++;
            enqueue_var(C, x);
            if (propagate(C, child, chg)) { C->st.fails++; continue; }
            dfs(C, child, depth + 1, chg);
        }
        free(child);
        return;
    }
    for (int v = 0; v < C->P->dsize[x] && !C->stop; ++v) {
        if (!D[(int64_t)x * C->dmax + v]) continue;
        if (C->max_nodes > 0 && C->st.nodes >= C->max_nodes) { C->stop = 3; break; }
        memcpy(child, D, bytes);
        memset(child + (int64_t)x * C->dmax, 0, (size_t)C->dmax);
        child[(int64_t)x * C->dmax + v] = 1;
        C->st.nodes++;
        enqueue_var(C, x);
        if (propagate(C, child, chg)) { C->st.fails++; continue; }
        dfs(C, child, depth + 1, chg);
    }
    free(child);
}

static int setup(ctx_t *C, const orc_problem *P) {
    memset(C, 0, sizeof(*C));
    C->P = P;
    C->n = P->n;
    C->dmax = 1;
    for (int i = 0; i < P->n; ++i) {
        if (P->dsize[i] < 1) return -1;
        if (P->dsize[i] > C->dmax) C->dmax = P->dsize[i];
    }
    C->W = (C->dmax + 31) / 32;
    C->prop = (prop_t *)malloc(sizeof(prop_t) * (size_t)(2 * P->m + 1));
    for (int c = 0; c < P->m; ++c) {
        int ty = P->type[c], k = P->arity[c];
        const int32_t *sc = P->vars + P->var_off[c];
        for (int t = 0; t < k; ++t)
            if (sc[t] < 0 || sc[t] >= P->n) return -1;
        if (ty == T_UNARY) {
            if (k != 1) return -1;
        } else if (ty >= T_TABLE2 && ty <= T_QUEENS) {
            if (k != 2 || sc[0] == sc[1]) return -1;
            C->prop[C->nprop].con = c; C->prop[C->nprop].dir = 0; C->nprop++;
            C->prop[C->nprop].con = c; C->prop[C->nprop].dir = 1; C->nprop++;
        } else if (ty == T_ALLDIFF || ty == T_LINEAR || ty == T_ALLDIFF_GAC || ty == T_LINEAR_AD) {
            if (k < 1) return -1;
            if (ty == T_ALLDIFF_GAC || ty == T_LINEAR_AD)  /* a scope is a set of variables */
                for (int t = 0; t < k; ++t)
                    for (int u = t + 1; u < k; ++u)
                        if (sc[t] == sc[u]) return -1;
            if (ty == T_LINEAR || ty == T_LINEAR_AD)
                for (int t = 0; t < k; ++t)
                    if (P->params[P->par_off[c] + 1 + t] <= 0) return -1;
            C->prop[C->nprop].con = c; C->prop[C->nprop].dir = 0; C->nprop++;
        } else {
            return -1;
        }
    }
    /* watch lists: every propagator whose constraint scope contains v */
    C->watch_off = (int *)calloc((size_t)P->n + 1, sizeof(int));
    for (int p = 0; p < C->nprop; ++p) {
        int c = C->prop[p].con;
        for (int64_t t = P->var_off[c]; t < P->var_off[c + 1]; ++t) C->watch_off[P->vars[t] + 1]++;
    }
    for (int v = 0; v < P->n; ++v) C->watch_off[v + 1] += C->watch_off[v];
    C->watch = (int *)malloc(sizeof(int) * (size_t)(C->watch_off[P->n] + 1));
    int *fill = (int *)calloc((size_t)P->n + 1, sizeof(int));
    for (int p = 0; p < C->nprop; ++p) {
        int c = C->prop[p].con;
        for (int64_t t = P->var_off[c]; t < P->var_off[c + 1]; ++t) {
            int v = P->vars[t];
            C->watch[C->watch_off[v] + fill[v]++] = p;
        }
    }
    free(fill);
    C->qcap = C->nprop + 1;
    C->queue = (int *)malloc(sizeof(int) * (size_t)C->qcap);
    C->inq = (unsigned char *)calloc((size_t)C->nprop + 1, 1);
    return 0;
}

static void teardown(ctx_t *C) {
    free(C->prop); free(C->watch_off); free(C->watch); free(C->queue); free(C->inq);
}

/* initial domains: the declared ranges, the optional init bits, and the
   unary constraints (node consistency) */
static void initial_domains(ctx_t *C, unsigned char *D) {
    const orc_problem *P = C->P;
    memset(D, 0, (size_t)C->n * (size_t)C->dmax);
    for (int i = 0; i < C->n; ++i)
        for (int a = 0; a < P->dsize[i]; ++a) {
            int ok = 1;
            if (P->init) ok = (P->init[(int64_t)i * C->W + a / 32] >> (a % 32)) & 1u;
            D[(int64_t)i * C->dmax + a] = (unsigned char)ok;
        }
    for (int c = 0; c < P->m; ++c) {
        if (P->type[c] != T_UNARY) continue;
        int x = P->vars[P->var_off[c]];
        const uint32_t *t = P->tabs + P->tab_off[c];
        for (int a = 0; a < P->dsize[x]; ++a)
            if (!((t[a / 32] >> (a % 32)) & 1u)) D[(int64_t)x * C->dmax + a] = 0;
    }
}

static int root_fixpoint(ctx_t *C, unsigned char *D, unsigned char *chg) {
    initial_domains(C, D);
    for (int i = 0; i < C->n; ++i)
        if (dom_size(C, D, i) == 0) return 1;
    for (int p = 0; p < C->nprop; ++p) enqueue(C, p);
    return propagate(C, D, chg);
}

/* ------------------------------------------------------------ exported */

/* Full search.  mode: 0 first, 1 all (store up to sol_cap), 2 count.
   max_nodes / cap: 0 = unlimited.  two_way: 2-way branching (x = min D_x,
   then x != min D_x) instead of one child per value.  Returns 0, or -1 on
   malformed input. */
int orc_solve2(const orc_problem *P, int mode, int64_t max_nodes, int64_t cap,
               int32_t *sols, int64_t sol_cap, int two_way, orc_stats *out) {
    ctx_t C;
    if (setup(&C, P)) { teardown(&C); return -1; }
    C.mode = mode;
    C.two_way = two_way != 0;
    C.max_nodes = max_nodes;
    C.cap = cap;
    C.sols = sols;
    C.sol_cap = sols ? sol_cap : 0;
    size_t bytes = (size_t)(C.n > 0 ? C.n : 1) * (size_t)C.dmax;
    unsigned char *D = (unsigned char *)malloc(bytes);
    unsigned char *chg = (unsigned char *)malloc((size_t)(C.n > 0 ? C.n : 1));
    C.st.nodes = 1;
    if (root_fixpoint(&C, D, chg)) {
        C.st.fails = 1;
    } else {
        dfs(&C, D, 0, chg);
    }
    if (C.stop == 2 || C.stop == 3) C.st.verdict = V_LIMIT;
    else C.st.verdict = C.st.count > 0 ? V_SAT : V_UNSAT;
    *out = C.st;
    free(D); free(chg);
    teardown(&C);
    return 0;
}

/* d-way labeling (the default reading). */
int orc_solve(const orc_problem *P, int mode, int64_t max_nodes, int64_t cap,
              int32_t *sols, int64_t sol_cap, orc_stats *out) {
    return orc_solve2(P, mode, max_nodes, cap, sols, sol_cap, 0, out);
}

/* Root fixpoint as n x W bit words (bit a = value lo_i + a).
   Returns 0 (consistent), 1 (failed) or -1 (malformed). */
int orc_root(const orc_problem *P, uint32_t *out_bits, int64_t *revisions) {
    ctx_t C;
    if (setup(&C, P)) { teardown(&C); return -1; }
    size_t bytes = (size_t)(C.n > 0 ? C.n : 1) * (size_t)C.dmax;
    unsigned char *D = (unsigned char *)malloc(bytes);
    unsigned char *chg = (unsigned char *)malloc((size_t)(C.n > 0 ? C.n : 1));
    int r = root_fixpoint(&C, D, chg);
    memset(out_bits, 0, sizeof(uint32_t) * (size_t)C.n * (size_t)C.W);
    for (int i = 0; i < C.n; ++i)
        for (int a = 0; a < P->dsize[i]; ++a)
            if (D[(int64_t)i * C.dmax + a]) out_bits[(int64_t)i * C.W + a / 32] |= 1u << (a % 32);
    if (revisions) *revisions = C.st.revisions;
    free(D); free(chg);
    teardown(&C);
    return r;
}

/* Direct check of one assignment (values, not indices) against the initial
   domains and every constraint's definition.  1 = solution, 0 = not. */
int orc_verify(const orc_problem *P, const int32_t *x) {
    int dmax = 1;
    for (int i = 0; i < P->n; ++i)
        if (P->dsize[i] > dmax) dmax = P->dsize[i];
    int W = (dmax + 31) / 32;
    for (int i = 0; i < P->n; ++i) {
        int64_t a = (int64_t)x[i] - P->lo[i];
        if (a < 0 || a >= P->dsize[i]) return 0;
        if (P->init && !((P->init[(int64_t)i * W + a / 32] >> (a % 32)) & 1u)) return 0;
    }
    for (int c = 0; c < P->m; ++c) {
        const int32_t *sc = P->vars + P->var_off[c];
        const int64_t *par = P->params + P->par_off[c];
        const uint32_t *t = P->tabs + P->tab_off[c];
        int k = P->arity[c];
        switch (P->type[c]) {
        case T_UNARY: {
            int64_t a = (int64_t)x[sc[0]] - P->lo[sc[0]];
            if (!((t[a / 32] >> (a % 32)) & 1u)) return 0;
            break;
        }
        case T_TABLE2: {
            int64_t a = (int64_t)x[sc[0]] - P->lo[sc[0]], b = (int64_t)x[sc[1]] - P->lo[sc[1]];
            int Wj = (P->dsize[sc[1]] + 31) / 32;
            if (!((t[a * Wj + b / 32] >> (b % 32)) & 1u)) return 0;
            break;
        }
        case T_NEQ:
            if (!((int64_t)x[sc[0]] != (int64_t)x[sc[1]] + par[0])) return 0;
            break;
        case T_LT:
            if (!((int64_t)x[sc[0]] < (int64_t)x[sc[1]] + par[0])) return 0;
            break;
        case T_QUEENS: {
            int64_t d = (int64_t)x[sc[0]] - x[sc[1]];
            if (d == 0 || d == par[0] || -d == par[0]) return 0;
            break;
        }
        case T_ALLDIFF:
        case T_ALLDIFF_GAC:
            for (int u = 0; u < k; ++u)
                for (int w = u + 1; w < k; ++w)
                    if (x[sc[u]] == x[sc[w]]) return 0;
            break;
        case T_LINEAR:
        case T_LINEAR_AD: {
            int64_t s = 0;
            for (int u = 0; u < k; ++u) s += par[1 + u] * (int64_t)x[sc[u]];
            if (s > par[0]) return 0;
            break;
        }
        default:
            return 0;
        }
    }
    return 1;
}

/* Brute force: walk every assignment of the declared domains (odometer) and
   keep those orc_verify accepts.  Stores up to sol_cap solutions in
   enumeration order.  Returns the count, or -1 if the product of the domain
   sizes exceeds limit. */
int64_t orc_brute(const orc_problem *P, int64_t limit, int32_t *sols, int64_t sol_cap) {
    double prod = 1.0;
    for (int i = 0; i < P->n; ++i) prod *= (double)P->dsize[i];
    if (prod > (double)limit) return -1;
    int32_t *x = (int32_t *)malloc(sizeof(int32_t) * (size_t)(P->n > 0 ? P->n : 1));
    for (int i = 0; i < P->n; ++i) x[i] = P->lo[i];
    int64_t count = 0;
    for (;;) {
        if (orc_verify(P, x)) {
            if (sols && count < sol_cap) memcpy(sols + count * P->n, x, sizeof(int32_t) * (size_t)P->n);
            ++count;
        }
        int i = P->n - 1;
        while (i >= 0) {
            if (x[i] < P->lo[i] + P->dsize[i] - 1) { x[i]++; break; }
            x[i] = P->lo[i];
            --i;
        }
        if (i < 0) break;
    }
    free(x);
    return count;
}
