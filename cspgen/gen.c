/*
 * Seeded synthetic CSP instance generators.
 *
 * This module only draws random instances; it contains none of the solving
 * method (no propagation, no search, no verification).  Both the CPU oracle
 * and the GPU solver consume its output, which is a flat constraint list:
 *
 *   n variables; variable i takes values lo[i] .. lo[i]+dsize[i]-1.
 *   m constraints; constraint c has type[c], arity[c], scope
 *   vars[var_off[c] .. var_off[c+1]), integer parameters
 *   params[par_off[c] .. par_off[c+1]) and packed bit rows
 *   tabs[tab_off[c] .. tab_off[c+1]).
 *
 * Type codes and their parameters:
 *   0 UNARY      scope (i);    tabs = ceil(d_i/32) words, bit a = value lo_i+a allowed
 *   1 TABLE2     scope (i,j);  tabs = d_i rows of ceil(d_j/32) words; bit b of row a
 *                              set iff (lo_i+a, lo_j+b) is an allowed pair
 *   2 NEQ        scope (i,j);  params {off}: x_i != x_j + off
 *   3 LT         scope (i,j);  params {off}: x_i <  x_j + off
 *   4 QUEENS     scope (i,j);  params {k}:   x_i != x_j and |x_i - x_j| != k
 *   5 ALLDIFF    scope (v_0..v_{k-1}): pairwise different values
 *   6 LINEAR_LE  scope (v_0..v_{k-1}); params {b, a_0..a_{k-1}}: sum a_t x_{v_t} <= b
 *
 * Random numbers: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014).  A uniform
 * integer in [0, r) rejects draws from the top 2^64 mod r values.  Choosing s
 * of N items without replacement is a partial Fisher-Yates shuffle.  The seed
 * of instance `index` in a family with base seed B is B ^ (index * golden64).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN64 0x9E3779B97F4A7C15ULL

typedef struct {
    int32_t n;
    int32_t m;
    int32_t *lo;
    int32_t *dsize;
    int32_t *type;
    int32_t *arity;
    int64_t *var_off;
    int32_t *vars;
    int64_t *par_off;
    int64_t *params;
    int64_t *tab_off;
    uint32_t *tabs;
    /* capacities (private) */
    int64_t cap_m, cap_vars, cap_par, cap_tab;
} gen_inst;

/* ---------------------------------------------------------------- RNG */
typedef struct { uint64_t s; } sm64;

static uint64_t sm64_next(sm64 *r) {
    uint64_t z = (r->s += GOLDEN64);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform integer in [0, r), r >= 1 */
static uint64_t sm64_below(sm64 *g, uint64_t r) {
    uint64_t rem = (0 - r) % r; /* 2^64 mod r */
    uint64_t lim = 0 - rem;     /* accept x < lim (lim == 0 means all) */
    for (;;) {
        uint64_t x = sm64_next(g);
        if (rem == 0 || x < lim) return x % r;
    }
}

static int64_t sm64_range(sm64 *g, int64_t lo, int64_t hi) { /* inclusive */
    return lo + (int64_t)sm64_below(g, (uint64_t)(hi - lo + 1));
}

/* choose s distinct of 0..N-1 in pick order (partial Fisher-Yates) */
static void pick_without_replacement(sm64 *g, int64_t N, int64_t s, int64_t *scratch, int64_t *out) {
    for (int64_t i = 0; i < N; ++i) scratch[i] = i;
    for (int64_t k = 0; k < s; ++k) {
        int64_t r = k + (int64_t)sm64_below(g, (uint64_t)(N - k));
        int64_t t = scratch[k]; scratch[k] = scratch[r]; scratch[r] = t;
        out[k] = scratch[k];
    }
}

uint64_t gen_instance_seed(uint64_t base, uint64_t index) { return base ^ (index * GOLDEN64); }

/* exported for the generator's own determinism tests */
void gen_rng_stream(uint64_t seed, int64_t count, uint64_t *out) {
    sm64 g = {seed};
    for (int64_t i = 0; i < count; ++i) out[i] = sm64_next(&g);
}
void gen_rng_below(uint64_t seed, uint64_t r, int64_t count, uint64_t *out) {
    sm64 g = {seed};
    for (int64_t i = 0; i < count; ++i) out[i] = sm64_below(&g, r);
}

/* ------------------------------------------------------------ builder */
static void *xgrow(void *p, int64_t *cap, int64_t need, size_t elt) {
    if (need <= *cap) return p;
    int64_t c = *cap ? *cap : 16;
    while (c < need) c *= 2;
    void *q = realloc(p, (size_t)c * elt);
    if (!q) abort();
    *cap = c;
    return q;
}

static gen_inst *inst_new(int n) {
    gen_inst *I = (gen_inst *)calloc(1, sizeof(gen_inst));
    I->n = n;
    I->lo = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    I->dsize = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    I->cap_m = 16;
    I->type = (int32_t *)malloc(16 * sizeof(int32_t));
    I->arity = (int32_t *)malloc(16 * sizeof(int32_t));
    I->var_off = (int64_t *)calloc(17, sizeof(int64_t));
    I->par_off = (int64_t *)calloc(17, sizeof(int64_t));
    I->tab_off = (int64_t *)calloc(17, sizeof(int64_t));
    return I;
}

static void inst_reserve_m(gen_inst *I, int64_t need) {
    if (need <= I->cap_m) return;
    int64_t c = I->cap_m;
    while (c < need) c *= 2;
    I->type = (int32_t *)realloc(I->type, (size_t)c * sizeof(int32_t));
    I->arity = (int32_t *)realloc(I->arity, (size_t)c * sizeof(int32_t));
    I->var_off = (int64_t *)realloc(I->var_off, (size_t)(c + 1) * sizeof(int64_t));
    I->par_off = (int64_t *)realloc(I->par_off, (size_t)(c + 1) * sizeof(int64_t));
    I->tab_off = (int64_t *)realloc(I->tab_off, (size_t)(c + 1) * sizeof(int64_t));
    if (!I->type || !I->arity || !I->var_off || !I->par_off || !I->tab_off) abort();
    I->cap_m = c;
}

/* append a constraint; returns pointer to its (zeroed) table words */
static uint32_t *inst_add(gen_inst *I, int type, int arity, const int32_t *vars,
                          int npar, const int64_t *par, int64_t ntab) {
    int64_t c = I->m;
    inst_reserve_m(I, c + 2);
    I->type[c] = type;
    I->arity[c] = arity;
    int64_t v0 = I->var_off[c], p0 = I->par_off[c], t0 = I->tab_off[c];
    I->vars = (int32_t *)xgrow(I->vars, &I->cap_vars, v0 + arity, sizeof(int32_t));
    I->params = (int64_t *)xgrow(I->params, &I->cap_par, p0 + npar, sizeof(int64_t));
    I->tabs = (uint32_t *)xgrow(I->tabs, &I->cap_tab, t0 + ntab, sizeof(uint32_t));
    for (int k = 0; k < arity; ++k) I->vars[v0 + k] = vars[k];
    for (int k = 0; k < npar; ++k) I->params[p0 + k] = par[k];
    memset(I->tabs + t0, 0, (size_t)ntab * sizeof(uint32_t));
    I->var_off[c + 1] = v0 + arity;
    I->par_off[c + 1] = p0 + npar;
    I->tab_off[c + 1] = t0 + ntab;
    I->m = (int32_t)(c + 1);
    return I->tabs + t0;
}

static int wordsof(int d) { return (d + 31) / 32; }

void gen_free(gen_inst *I) {
    if (!I) return;
    free(I->lo); free(I->dsize); free(I->type); free(I->arity);
    free(I->var_off); free(I->vars); free(I->par_off); free(I->params);
    free(I->tab_off); free(I->tabs);
    free(I);
}

/* ------------------------------------------------------------ families */

/* n-queens: x_i = row of the queen in column i, values 1..n;
   one combined pair constraint per column pair with k = j - i. */
gen_inst *gen_queens(int n) {
    gen_inst *I = inst_new(n);
    for (int i = 0; i < n; ++i) { I->lo[i] = 1; I->dsize[i] = n; }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            int32_t sc[2] = {i, j};
            int64_t k = j - i;
            inst_add(I, 4, 2, sc, 1, &k, 0);
        }
    return I;
}

/* The two-variable example of the paper's introduction (Sec. 1.1):
   x1 in 1..5, x2 in 1..10, c1 = {x1 > 3} as a unary set, c2 = {x1 < x2}
   either as its set of allowed pairs over the original domains (form 0)
   or as the arithmetic LT constraint (form 1). */
gen_inst *gen_worked_example(int form) {
    gen_inst *I = inst_new(2);
    I->lo[0] = 1; I->dsize[0] = 5;
    I->lo[1] = 1; I->dsize[1] = 10;
    int32_t s0[1] = {0};
    uint32_t *u = inst_add(I, 0, 1, s0, 0, NULL, 1);
    for (int a = 0; a < 5; ++a)
        if (1 + a > 3) u[0] |= 1u << a;
    int32_t s01[2] = {0, 1};
    if (form == 0) {
        uint32_t *t = inst_add(I, 1, 2, s01, 0, NULL, 5 * 1);
        for (int a = 0; a < 5; ++a)
            for (int b = 0; b < 10; ++b)
                if (1 + a < 1 + b) t[a] |= 1u << b;
    } else {
        int64_t off = 0;
        inst_add(I, 3, 2, s01, 1, &off, 0);
    }
    return I;
}

/* Random binary CSP with exactly m constrained pairs and exactly t forbidden
   value pairs per table (model-RB style exact tightness).  m and t are given
   as per-mille of C(n,2) and d^2, rounded half up in integer arithmetic. */
static void add_random_tables(gen_inst *I, sm64 *g, int n, int d, int64_t m, int64_t t) {
    int64_t P = (int64_t)n * (n - 1) / 2;
    int64_t *pi = (int64_t *)malloc((size_t)P * sizeof(int64_t));
    int64_t *pj = (int64_t *)malloc((size_t)P * sizeof(int64_t));
    int64_t q = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) { pi[q] = i; pj[q] = j; ++q; }
    int64_t *scratch = (int64_t *)malloc((size_t)(P > (int64_t)d * d ? P : (int64_t)d * d) * sizeof(int64_t));
    int64_t *chosen = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    pick_without_replacement(g, P, m, scratch, chosen);
    int64_t D2 = (int64_t)d * d;
    int64_t *cells = (int64_t *)malloc((size_t)(t > 0 ? t : 1) * sizeof(int64_t));
    int W = wordsof(d);
    for (int64_t c = 0; c < m; ++c) {
        int32_t sc[2] = {(int32_t)pi[chosen[c]], (int32_t)pj[chosen[c]]};
        uint32_t *tab = inst_add(I, 1, 2, sc, 0, NULL, (int64_t)d * W);
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) tab[(int64_t)a * W + b / 32] |= 1u << (b % 32);
        pick_without_replacement(g, D2, t, scratch, cells);
        for (int64_t k = 0; k < t; ++k) {
            int64_t a = cells[k] / d, b = cells[k] % d;
            tab[a * W + b / 32] &= ~(1u << (b % 32));
        }
    }
    free(pi); free(pj); free(scratch); free(chosen); free(cells);
}

gen_inst *gen_rb(uint64_t seed, int n, int d, int dens_pm, int tight_pm) {
    gen_inst *I = inst_new(n);
    for (int i = 0; i < n; ++i) { I->lo[i] = 0; I->dsize[i] = d; }
    sm64 g = {seed};
    int64_t P = (int64_t)n * (n - 1) / 2;
    int64_t m = ((int64_t)dens_pm * P + 500) / 1000;
    int64_t t = ((int64_t)tight_pm * d * d + 500) / 1000;
    add_random_tables(I, &g, n, d, m, t);
    return I;
}

/* One instance of the batched sweep: n ~ U{nlo..nhi}, d ~ U{dlo..dhi},
   density per-mille ~ U{plo..phi}, tightness per-mille ~ U{tlo..thi},
   drawn in that order from the instance's own stream. */
gen_inst *gen_rb_sweep(uint64_t seed, int nlo, int nhi, int dlo, int dhi,
                       int plo, int phi, int tlo, int thi) {
    sm64 g = {seed};
    int n = (int)sm64_range(&g, nlo, nhi);
    int d = (int)sm64_range(&g, dlo, dhi);
    int dens = (int)sm64_range(&g, plo, phi);
    int tight = (int)sm64_range(&g, tlo, thi);
    gen_inst *I = inst_new(n);
    for (int i = 0; i < n; ++i) { I->lo[i] = 0; I->dsize[i] = d; }
    int64_t P = (int64_t)n * (n - 1) / 2;
    int64_t m = ((int64_t)dens * P + 500) / 1000;
    int64_t t = ((int64_t)tight * d * d + 500) / 1000;
    add_random_tables(I, &g, n, d, m, t);
    return I;
}

/* Tree-structured binary CSP: variable i >= 1 is constrained with a parent
   drawn uniformly from 0..i-1; every table forbids exactly t pairs. */
gen_inst *gen_tree(uint64_t seed, int n, int d, int tight_pm) {
    gen_inst *I = inst_new(n);
    for (int i = 0; i < n; ++i) { I->lo[i] = 0; I->dsize[i] = d; }
    sm64 g = {seed};
    int64_t D2 = (int64_t)d * d;
    int64_t t = ((int64_t)tight_pm * D2 + 500) / 1000;
    int64_t *scratch = (int64_t *)malloc((size_t)D2 * sizeof(int64_t));
    int64_t *cells = (int64_t *)malloc((size_t)(t > 0 ? t : 1) * sizeof(int64_t));
    int W = wordsof(d);
    for (int i = 1; i < n; ++i) {
        int p = (int)sm64_below(&g, (uint64_t)i);
        int32_t sc[2] = {p, i};
        uint32_t *tab = inst_add(I, 1, 2, sc, 0, NULL, (int64_t)d * W);
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) tab[(int64_t)a * W + b / 32] |= 1u << (b % 32);
        pick_without_replacement(&g, D2, t, scratch, cells);
        for (int64_t k = 0; k < t; ++k) {
            int64_t a = cells[k] / d, b = cells[k] % d;
            tab[a * W + b / 32] &= ~(1u << (b % 32));
        }
    }
    free(scratch); free(cells);
    return I;
}

/* Global-constraint family: n vars over lo..lo+d-1; n_ad all-different
   constraints over k_ad distinct vars each (subsets drawn independently);
   n_lin linear constraints sum a_t x_t <= b with a_t ~ U{1..amax} over either
   all n vars (lin_k <= 0) or lin_k distinct vars; b = floor(b_pm * hi * sum(a) / 1000)
   with hi = lo + d - 1 the largest value (b_pm = 450: 45% of the maximum sum). */
gen_inst *gen_global(uint64_t seed, int n, int lo, int d, int n_ad, int k_ad,
                     int n_lin, int lin_k, int amax, int b_pm) {
    gen_inst *I = inst_new(n);
    for (int i = 0; i < n; ++i) { I->lo[i] = lo; I->dsize[i] = d; }
    sm64 g = {seed};
    int64_t *scratch = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *pick = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int32_t *sc = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *par = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    for (int c = 0; c < n_ad; ++c) {
        pick_without_replacement(&g, n, k_ad, scratch, pick);
        for (int t = 0; t < k_ad; ++t) sc[t] = (int32_t)pick[t];
        inst_add(I, 5, k_ad, sc, 0, NULL, 0);
    }
    int hi = lo + d - 1;
    for (int c = 0; c < n_lin; ++c) {
        int k = (lin_k <= 0 || lin_k > n) ? n : lin_k;
        if (k == n) {
            for (int t = 0; t < n; ++t) sc[t] = t;
        } else {
            pick_without_replacement(&g, n, k, scratch, pick);
            for (int t = 0; t < k; ++t) sc[t] = (int32_t)pick[t];
        }
        int64_t sum = 0;
        for (int t = 0; t < k; ++t) { par[1 + t] = sm64_range(&g, 1, amax); sum += par[1 + t]; }
        int64_t maxsum = sum * (int64_t)hi;
        int64_t num = (int64_t)b_pm * maxsum;
        par[0] = num >= 0 ? num / 1000 : -((-num + 999) / 1000);
        inst_add(I, 6, k, sc, 1 + k, par, 0);
    }
    free(scratch); free(pick); free(sc); free(par);
    return I;
}

/* Small random instances mixing every constraint type, for brute-force
   comparison.  Domains: d_i ~ U{1..dmax}, lo_i ~ U{-2..2}. */
gen_inst *gen_mixed(uint64_t seed, int n, int dmax, int m, int type_mask) {
    gen_inst *I = inst_new(n);
    sm64 g = {seed};
    for (int i = 0; i < n; ++i) {
        I->dsize[i] = (int32_t)sm64_range(&g, 1, dmax);
        I->lo[i] = (int32_t)sm64_range(&g, -2, 2);
    }
    int64_t *scratch = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *pick = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int32_t sc[64];
    int64_t par[65];
    int types[7], nt = 0;
    for (int t = 0; t < 7; ++t)
        if (type_mask & (1 << t)) types[nt++] = t;
    for (int c = 0; c < m && nt > 0; ++c) {
        int ty = types[sm64_below(&g, (uint64_t)nt)];
        if (ty != 0 && n < 2) ty = 0;
        if (n < 1) break;
        if (ty == 0) {
            int i = (int)sm64_below(&g, (uint64_t)n);
            sc[0] = i;
            int W = wordsof(I->dsize[i]);
            uint32_t *t = inst_add(I, 0, 1, sc, 0, NULL, W);
            for (int a = 0; a < I->dsize[i]; ++a)
                if (sm64_below(&g, 1000) < 700) t[a / 32] |= 1u << (a % 32);
        } else if (ty >= 1 && ty <= 4) {
            pick_without_replacement(&g, n, 2, scratch, pick);
            sc[0] = (int32_t)pick[0]; sc[1] = (int32_t)pick[1];
            if (ty == 1) {
                int di = I->dsize[sc[0]], dj = I->dsize[sc[1]], W = wordsof(dj);
                uint32_t *t = inst_add(I, 1, 2, sc, 0, NULL, (int64_t)di * W);
                for (int a = 0; a < di; ++a)
                    for (int b = 0; b < dj; ++b)
                        if (sm64_below(&g, 1000) < 650) t[(int64_t)a * W + b / 32] |= 1u << (b % 32);
            } else if (ty == 2) {
                par[0] = sm64_range(&g, -2, 2);
                inst_add(I, 2, 2, sc, 1, par, 0);
            } else if (ty == 3) {
                par[0] = sm64_range(&g, -1, 3);
                inst_add(I, 3, 2, sc, 1, par, 0);
            } else {
                par[0] = sm64_range(&g, 1, 3);
                inst_add(I, 4, 2, sc, 1, par, 0);
            }
        } else {
            int kmax = n < 5 ? n : 5;
            int k = (int)sm64_range(&g, 2, kmax);
            pick_without_replacement(&g, n, k, scratch, pick);
            for (int t = 0; t < k; ++t) sc[t] = (int32_t)pick[t];
            if (ty == 5) {
                inst_add(I, 5, k, sc, 0, NULL, 0);
            } else {
                int64_t lo_sum = 0, hi_sum = 0;
                for (int t = 0; t < k; ++t) {
                    par[1 + t] = sm64_range(&g, 1, 4);
                    lo_sum += par[1 + t] * I->lo[sc[t]];
                    hi_sum += par[1 + t] * (I->lo[sc[t]] + I->dsize[sc[t]] - 1);
                }
                par[0] = sm64_range(&g, lo_sum, hi_sum);
                inst_add(I, 6, k, sc, 1 + k, par, 0);
            }
        }
    }
    free(scratch); free(pick);
    return I;
}
