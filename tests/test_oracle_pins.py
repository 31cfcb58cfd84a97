"""Pins of the CPU oracle against facts that do not come from the oracle:
the paper's worked example (Sec. 1.1), n-queens counts (OEIS A000170),
exhaustive enumeration, closed-form counts, tree-CSP counts by dynamic
programming, and projections that arc consistency must reach exactly."""
import itertools
import math
import os

import numpy as np
import pytest

import cspgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows[parts[0]] = [int(x) for x in parts[1:]]
    return rows


def _bits_to_values(inst, bits):
    out = []
    for i in range(inst.n):
        vals = [int(inst.lo[i]) + a for a in range(int(inst.dsize[i]))
                if (int(bits[i][a // 32]) >> (a % 32)) & 1]
        out.append(vals)
    return out


def _canon(sols):
    return sorted(tuple(int(v) for v in row) for row in sols)


# ----------------------------------------------------------- worked example

@pytest.mark.parametrize("form", [0, 1])
def test_worked_example(form):
    g = _read_golden("worked_example.txt")
    inst = cspgen.worked_example(form)
    # the printed extension of c1 (unary set over D1)
    c1 = [int(inst.lo[0]) + a for a in range(5) if (int(inst.tab(0)[0]) >> a) & 1]
    assert c1 == g["c1_extension"]
    if form == 0:
        # the printed extension of c2: all (a, b) with a < b over the original domains
        tab = inst.tab(1)
        pairs = [(1 + a, 1 + b) for a in range(5) for b in range(10) if (int(tab[a]) >> b) & 1]
        assert len(pairs) == g["c2_pairs"][0]
        assert pairs[0] == (1, 2) and pairs[-1] == (5, 10)
        assert all(a < b for a, b in pairs)
    failed, bits, _ = oracle.root(inst)
    assert not failed
    D = _bits_to_values(inst, bits)
    assert D[0] == g["root_D1"] and D[1] == g["root_D2"]
    r = oracle.solve(inst, oracle.MODE_ALL, sol_cap=64)
    assert r.verdict == "SAT" and r.count == g["count"][0]
    assert r.nodes == g["nodes"][0] and r.fails == g["fails"][0]
    cnt, bsols = oracle.brute(inst, sol_cap=64)
    assert cnt == g["count"][0]
    assert _canon(r.solutions) == _canon(bsols)
    f = oracle.solve(inst, oracle.MODE_FIRST, sol_cap=1)
    assert f.verdict == "SAT" and f.solutions[0].tolist() == g["first"]
    t = oracle.solve(inst, oracle.MODE_ALL, sol_cap=64, two_way=True)
    assert t.count == g["count"][0] and _canon(t.solutions) == _canon(bsols)
    assert t.nodes == g["nodes_two_way"][0] and t.fails == 0


# ------------------------------------------------------------------ queens

def test_nqueens_counts():
    g = _read_golden("nqueens_counts.txt")
    for n in range(1, 11):
        r = oracle.solve(cspgen.queens(n), oracle.MODE_COUNT)
        assert r.count == g[str(n)][0], n
        assert r.verdict == ("SAT" if r.count else "UNSAT")


def test_8queens_solution_set_symmetry_and_brute():
    inst = cspgen.queens(8)
    r = oracle.solve(inst, oracle.MODE_ALL, sol_cap=200)
    assert r.count == 92 and r.n_written == 92
    sols = set(_canon(r.solutions))
    assert len(sols) == 92
    n = 8

    def sym(s):
        # board symmetries acting on (column, row) pairs with rows 1..n
        cells = [(c, s[c] - 1) for c in range(n)]
        outs = []
        for t in range(8):
            mapped = []
            for (c, rr) in cells:
                x, y = c, rr
                for _ in range(t % 4):
                    x, y = y, n - 1 - x
                if t >= 4:
                    x = n - 1 - x
                mapped.append((x, y))
            row = [0] * n
            for (x, y) in mapped:
                row[x] = y + 1
            outs.append(tuple(row))
        return outs

    for s in sols:
        for t in sym(s):
            assert t in sols
    for s in sols:
        assert oracle.verify(inst, np.array(s))


def test_nqueens_brute_small():
    for n in range(1, 7):
        inst = cspgen.queens(n)
        cnt, bs = oracle.brute(inst, sol_cap=100)
        r = oracle.solve(inst, oracle.MODE_ALL, sol_cap=100)
        assert cnt == r.count
        assert _canon(bs) == _canon(r.solutions)


# ------------------------------------------------------------- brute force

@pytest.mark.parametrize("mask", [0x7F, 0x02, 0x1C, 0x20, 0x40, 0x61])
def test_random_mixed_vs_brute(mask):
    for idx in range(120):
        inst = cspgen.mixed(idx + 1000 * mask, n=5, dmax=5, m=6, type_mask=mask)
        cnt, bs = oracle.brute(inst, sol_cap=4000)
        r = oracle.solve(inst, oracle.MODE_ALL, sol_cap=4000)
        assert r.count == cnt, (idx, mask)
        assert _canon(r.solutions) == _canon(bs), (idx, mask)
        f = oracle.solve(inst, oracle.MODE_FIRST, sol_cap=1)
        assert f.verdict == ("SAT" if cnt else "UNSAT")
        if cnt:
            assert oracle.verify(inst, f.solutions[0])
            # first solution in ascending d-way order is the lexicographically
            # first under the oracle's own variable order; it must be one of them
            assert tuple(f.solutions[0].tolist()) in set(_canon(bs))


def test_random_mixed_with_init_vs_brute():
    rng = np.random.default_rng(5)
    for idx in range(80):
        inst = cspgen.mixed(idx + 77, n=5, dmax=6, m=5)
        init = inst.full_init()
        for i in range(inst.n):
            for a in range(int(inst.dsize[i])):
                if rng.random() < 0.3:
                    init[i, a // 32] &= np.uint32(~(1 << (a % 32)) & 0xFFFFFFFF)
        sub = inst.with_init(init)
        cnt, bs = oracle.brute(sub, sol_cap=4000)
        r = oracle.solve(sub, oracle.MODE_ALL, sol_cap=4000)
        assert r.count == cnt and _canon(r.solutions) == _canon(bs)


# ----------------------------------------------------------- verifier cases

def test_verifier_hand_cases():
    w = cspgen.worked_example(0)
    assert oracle.verify(w, [4, 5]) and oracle.verify(w, [5, 10])
    assert not oracle.verify(w, [3, 5])      # c1
    assert not oracle.verify(w, [5, 5])      # c2
    assert not oracle.verify(w, [4, 11])     # outside D2
    q = cspgen.queens(4)
    assert oracle.verify(q, [2, 4, 1, 3])
    assert not oracle.verify(q, [1, 3, 2, 4])   # diagonal
    assert not oracle.verify(q, [2, 2, 4, 1])   # same row
    g = cspgen.global_twin(0)
    # an assignment violating the first all-different
    sc = g.scope(0)
    x = np.zeros(g.n, dtype=np.int32)
    for t, v in enumerate(sc):
        x[v] = t
    x[sc[1]] = x[sc[0]]
    assert not oracle.verify(g, x)


# ------------------------------------------------------------ closed forms

def _custom(n, lo, d, cons):
    """Instance from (type, scope, params, table-words) tuples."""
    var_off, vars_, par_off, params, tab_off, tabs = [0], [], [0], [], [0], []
    types, ar = [], []
    for (ty, sc, par, tb) in cons:
        types.append(ty); ar.append(len(sc))
        vars_ += list(sc); var_off.append(len(vars_))
        params += list(par); par_off.append(len(params))
        tabs += list(tb); tab_off.append(len(tabs))
    return cspgen.Instance(
        lo=np.array(lo, np.int32), dsize=np.array(d, np.int32),
        type=np.array(types, np.int32), arity=np.array(ar, np.int32),
        var_off=np.array(var_off, np.int64), vars=np.array(vars_, np.int32),
        par_off=np.array(par_off, np.int64), params=np.array(params, np.int64),
        tab_off=np.array(tab_off, np.int64), tabs=np.array(tabs, np.uint32))


def test_no_constraints_product():
    inst = _custom(4, [0, 3, -2, 1], [3, 1, 4, 2], [])
    r = oracle.solve(inst, oracle.MODE_COUNT)
    assert r.count == 3 * 1 * 4 * 2
    # with no propagation the d-way tree has 1 + 2 + 2*3 + 2*3*4 nodes
    # (first-fail order: sizes 2, 3, 4)
    assert r.nodes == 1 + 2 + 6 + 24 and r.fails == 0


def test_empty_problem_and_empty_domain():
    r = oracle.solve(_custom(0, [], [], []), oracle.MODE_ALL, sol_cap=4)
    assert r.count == 1 and r.nodes == 1 and r.verdict == "SAT"
    inst = _custom(2, [0, 0], [3, 3], [(2, (0, 1), (0,), ())])
    sub = inst.with_init(np.array([[0b101], [0]], np.uint32))
    r = oracle.solve(sub, oracle.MODE_COUNT)
    assert r.count == 0 and r.verdict == "UNSAT" and r.nodes == 1 and r.fails == 1


@pytest.mark.parametrize("k,s", [(2, 3), (3, 3), (3, 5), (4, 6), (5, 7), (6, 6)])
def test_alldiff_permutation_count(k, s):
    inst = _custom(k, [0] * k, [s] * k, [(5, tuple(range(k)), (), ())])
    r = oracle.solve(inst, oracle.MODE_COUNT)
    assert r.count == math.factorial(s) // math.factorial(s - k)
    assert r.fails == 0  # singleton elimination never fails here
    # Node count in closed form.  All domains stay equal: after j labelings
    # singleton elimination leaves s - j values to every unlabelled variable,
    # so first-fail labels the variables in index order and level j of the
    # tree holds s!/(s-j)! nodes.  The last level exists only if the last
    # variable still has two values (s > k); with s = k it is a singleton
    # once the other k - 1 are labelled, and those nodes are the solutions.
    # A propagator without singleton elimination would branch on s values at
    # every level and fail on the repeated ones.
    perm = [math.factorial(s) // math.factorial(s - j) for j in range(k + 1)]
    assert r.nodes == (sum(perm) if s > k else sum(perm[:k]))


@pytest.mark.parametrize("k", [2, 3, 5, 8])
def test_alldiff_pigeonhole_fails_at_root(k):
    # k variables sharing k-1 values: no solution, detected by the pigeonhole
    # test at the root without any search
    inst = _custom(k, [0] * k, [k - 1] * k, [(5, tuple(range(k)), (), ())])
    r = oracle.solve(inst, oracle.MODE_COUNT)
    assert r.count == 0 and r.nodes == 1 and r.fails == 1


def _sum_le_count(n, U, b):
    # number of (x_1..x_n) in {0..U}^n with sum <= b (inclusion-exclusion)
    tot = 0
    for j in range(n + 1):
        r = b - j * (U + 1)
        if r < 0:
            break
        tot += (-1) ** j * math.comb(n, j) * math.comb(r + n, n)
    return tot


@pytest.mark.parametrize("n,U,b", [(3, 4, 5), (4, 3, 7), (5, 2, 4), (2, 9, 12), (6, 1, 3)])
def test_sum_le_closed_form(n, U, b):
    inst = _custom(n, [0] * n, [U + 1] * n, [(6, tuple(range(n)), (b,) + (1,) * n, ())])
    r = oracle.solve(inst, oracle.MODE_COUNT)
    assert r.count == _sum_le_count(n, U, b)
    # bounds reasoning is exact for a single sum: the root domains are 0..min(U, b)
    failed, bits, _ = oracle.root(inst)
    D = _bits_to_values(inst, bits)
    assert all(Di == list(range(min(U, b) + 1)) for Di in D)


def _sum_le_tree_nodes(n, U, b):
    """Nodes of the first-fail d-way tree of sum x_i <= b over {0..U}^n under
    bounds reasoning, counted from the structure of the problem alone.
    Bounds reasoning is exact for one sum of non-negative variables: after
    labelling x_1..x_j with sum S every unlabelled domain is {0..min(U, b-S)}
    and every such value extends to a solution, so no node fails.  All
    unlabelled domains stay equal, so first-fail labels x_1, x_2, ... in
    index order, and a node branches unless its unlabelled domains are all
    singletons, i.e. unless S = b (or U = 0, or every variable is labelled).
    Level j therefore holds the prefixes (x_1..x_j) with sum <= b whose
    first j-1 values sum to less than b; counted by dynamic programming over
    the prefix sum.  (Propagation weaker than bounds consistency would fail
    on some children; none can be stronger.)"""
    if U == 0:
        return 1
    nodes = 1
    ways = {0: 1}  # prefix sum -> prefixes of the current level that branch
    for j in range(1, n + 1):
        nxt = {}
        for S, w in ways.items():
            if S >= b:
                continue  # all unlabelled domains are {0}: a leaf
            for v in range(0, min(U, b - S) + 1):
                nxt[S + v] = nxt.get(S + v, 0) + w
        nodes += sum(nxt.values())
        ways = nxt
    return nodes


@pytest.mark.parametrize("n,U,b", [(3, 4, 5), (4, 3, 7), (5, 2, 4), (2, 9, 12), (6, 1, 3), (4, 5, 30)])
def test_sum_le_node_count_closed_form(n, U, b):
    inst = _custom(n, [0] * n, [U + 1] * n, [(6, tuple(range(n)), (b,) + (1,) * n, ())])
    r = oracle.solve(inst, oracle.MODE_COUNT)
    assert r.fails == 0
    assert r.nodes == _sum_le_tree_nodes(n, U, b)


def _knapsack_count(coef, U, b):
    # number of x in prod {0..U_t} with sum coef_t x_t <= b, by DP over the sum
    ways = {0: 1}
    for a, u in zip(coef, U):
        nxt = {}
        for s, w in ways.items():
            for v in range(u + 1):
                t = s + a * v
                if t <= b:
                    nxt[t] = nxt.get(t, 0) + w
        ways = nxt
    return sum(ways.values())


def test_linear_knapsack_dp():
    rng = np.random.default_rng(3)
    for _ in range(25):
        n = int(rng.integers(1, 6))
        coef = [int(c) for c in rng.integers(1, 10, n)]
        U = [int(u) for u in rng.integers(0, 7, n)]
        b = int(rng.integers(0, sum(c * u for c, u in zip(coef, U)) + 2))
        inst = _custom(n, [0] * n, [u + 1 for u in U], [(6, tuple(range(n)), (b,) + tuple(coef), ())])
        assert oracle.solve(inst, oracle.MODE_COUNT).count == _knapsack_count(coef, U, b)


# ------------------------------------------------- projections of one constraint

def _projection(inst, sols):
    proj = [set() for _ in range(inst.n)]
    for s in sols:
        for i, v in enumerate(s):
            proj[i].add(int(v))
    return [sorted(p) for p in proj]


@pytest.mark.parametrize("ty", [1, 2, 3, 4, 6])
def test_single_constraint_root_is_projection(ty):
    """For one binary constraint (arc consistency) or one sum <= b with positive
    coefficients (bounds reasoning), the root fixpoint keeps exactly the values
    that occur in some solution."""
    mask = 1 << ty
    seen = 0
    for idx in range(200):
        inst = cspgen.mixed(idx + 31 * ty, n=4, dmax=6, m=1, type_mask=mask)
        cnt, bs = oracle.brute(inst, sol_cap=5000)
        failed, bits, _ = oracle.root(inst)
        if cnt == 0:
            # an empty projection: the root must fail
            assert failed
            continue
        seen += 1
        assert not failed
        assert _bits_to_values(inst, bits) == _projection(inst, bs)
    assert seen > 20


# ------------------------------------------------------------------ trees

def _tree_count(inst):
    """Exact count of a tree-structured binary CSP by dynamic programming
    over the tree (children before parents)."""
    n, d = inst.n, int(inst.dsize[0])
    W = (d + 31) // 32
    msg = np.ones((n, d), dtype=object)
    children = [[] for _ in range(n)]
    edge = {}
    for c in range(inst.m):
        p, i = (int(v) for v in inst.scope(c))
        children[p].append(i)
        edge[i] = (p, inst.tab(c).reshape(d, W))
    for i in range(n - 1, -1, -1):
        for ch in children[i]:
            _, tab = edge[ch]
            for a in range(d):
                msg[i, a] *= sum(msg[ch, b] for b in range(d) if (int(tab[a, b // 32]) >> (b % 32)) & 1)
    return int(sum(msg[0]))


@pytest.mark.parametrize("idx", range(6))
def test_tree_csp_count_and_backtrack_free(idx):
    inst = cspgen.tree(idx, n=9, d=4, tight_pm=400)
    r = oracle.solve(inst, oracle.MODE_COUNT)
    assert r.count == _tree_count(inst)
    # arc consistency makes tree-structured CSPs backtrack-free (Freuder 1982):
    # a search under it never meets a failed node
    assert r.fails == 0
    # and the root fixpoint is the projection of the solution set
    if r.count:
        cnt, bs = oracle.brute(inst, sol_cap=300000)
        failed, bits, _ = oracle.root(inst)
        assert _bits_to_values(inst, bits) == _projection(inst, bs)


# ------------------------------------------------------ independent search

def _def_fixpoint(inst, D):
    """Propagation written from the definitions in the paper's Sec. 1.1
    reading: a value stays in a binary constraint's variable iff some value of
    the other variable forms an allowed pair (checked through the verifier's
    arithmetic on concrete values); all-different and sum <= b by their rules.
    Repeat whole passes until nothing changes."""
    n = inst.n

    def allowed(c, vi, vj):
        x = np.array([0] * n, dtype=np.int32)
        i, j = (int(v) for v in inst.scope(c))
        ty = int(inst.type[c])
        if ty == 1:
            a, b = vi - int(inst.lo[i]), vj - int(inst.lo[j])
            Wj = (int(inst.dsize[j]) + 31) // 32
            return (int(inst.tab(c)[a * Wj + b // 32]) >> (b % 32)) & 1 == 1
        p = int(inst.par(c)[0])
        if ty == 2:
            return vi != vj + p
        if ty == 3:
            return vi < vj + p
        return vi != vj and abs(vi - vj) != p

    changed = True
    while changed:
        changed = False
        for c in range(inst.m):
            ty = int(inst.type[c])
            sc = [int(v) for v in inst.scope(c)]
            if ty in (1, 2, 3, 4):
                i, j = sc
                ni = {a for a in D[i] if any(allowed(c, a, b) for b in D[j])}
                nj = {b for b in D[j] if any(allowed(c, a, b) for a in D[i])}
                if ni != D[i] or nj != D[j]:
                    D[i], D[j] = ni, nj
                    changed = True
            elif ty == 5:
                for t in sc:
                    if len(D[t]) == 1:
                        (w,) = D[t]
                        for u in sc:
                            if u != t and w in D[u]:
                                D[u] = D[u] - {w}
                                changed = True
                if any(not D[u] for u in sc):
                    return None
                if len(set().union(*[D[u] for u in sc])) < len(sc):
                    return None
            elif ty == 7:
                # generalized arc consistency: a value stays iff it occurs in
                # some tuple of pairwise different values (enumerated)
                keep = [set() for _ in sc]
                for tup in itertools.product(*[sorted(D[u]) for u in sc]):
                    if len(set(tup)) == len(tup):
                        for q, v in enumerate(tup):
                            keep[q].add(v)
                for q, u in enumerate(sc):
                    if keep[q] != D[u]:
                        D[u] = keep[q]
                        changed = True
                if any(not D[u] for u in sc):
                    return None
            elif ty == 6:
                par = [int(v) for v in inst.par(c)]
                b, coef = par[0], par[1:]
                S = sum(a * min(D[u]) for a, u in zip(coef, sc))
                if S > b:
                    return None
                for a, u in zip(coef, sc):
                    rest = S - a * min(D[u])
                    keep = {v for v in D[u] if a * v + rest <= b}
                    if keep != D[u]:
                        D[u] = keep
                        changed = True
            elif ty == 8:
                r = _linear_ad_rule(inst, c, D)
                if r is None:
                    return None
                changed |= r
            if any(not D[u] for u in range(n)):
                return None
    return D


def _linear_ad_rule(inst, c, D):
    """sum a_t x_t <= b together with the all-different constraints inside
    its scope (constraint order, disjoint ones only).  A group's part of the
    sum is bounded below by its smallest value over every assignment of
    pairwise different values from the union of its domains (enumerated
    here), and by the sum of its minima; a value v of x_t goes when a_t v plus
    the bound of everything else exceeds b, the rest of t's group counted by
    its minima.  Returns None on failure, else whether a domain shrank."""
    sc = [int(v) for v in inst.scope(c)]
    par = [int(v) for v in inst.par(c)]
    b, coef = par[0], par[1:]
    grp = [-1] * len(sc)
    G = 0
    for c2 in range(inst.m):
        if int(inst.type[c2]) not in (5, 7) or G == 16:
            continue
        s2 = [int(v) for v in inst.scope(c2)]
        if all(u in sc and grp[sc.index(u)] < 0 for u in s2):
            for u in s2:
                grp[sc.index(u)] = G
            G += 1
    S = sum(a * min(D[u]) for a, u, g in zip(coef, sc, grp) if g < 0)
    delta = []
    for g in range(G):
        pos = [t for t in range(len(sc)) if grp[t] == g]
        union = sorted(set().union(*[D[sc[t]] for t in pos]))
        if len(union) < len(pos):
            return None
        Pg = sum(coef[t] * min(D[sc[t]]) for t in pos)
        Lg = min(sum(coef[t] * v for t, v in zip(pos, vals))
                 for vals in itertools.permutations(union, len(pos)))
        S += max(Pg, Lg)
        delta.append(max(Pg, Lg) - Pg)
    if S > b:
        return None
    changed = False
    for t, (a, u) in enumerate(zip(coef, sc)):
        rest = S - a * min(D[u]) - (delta[grp[t]] if grp[t] >= 0 else 0)
        keep = {v for v in D[u] if a * v + rest <= b}
        if keep != D[u]:
            D[u] = keep
            changed = True
    return changed


def _def_search(inst, two_way=False):
    """Independent first-fail search over _def_fixpoint, d-way or 2-way
    (x = min D_x, then x != min D_x): returns (count, nodes, fails)."""
    D0 = []
    for i in range(inst.n):
        vals = set(int(inst.lo[i]) + a for a in range(int(inst.dsize[i])))
        D0.append(vals)
    for c in range(inst.m):
        if int(inst.type[c]) == 0:
            i = int(inst.scope(c)[0])
            t = inst.tab(c)
            D0[i] = {v for v in D0[i] if (int(t[(v - int(inst.lo[i])) // 32]) >> ((v - int(inst.lo[i])) % 32)) & 1}
    stats = {"count": 0, "nodes": 1, "fails": 0}

    def rec(D):
        if all(len(x) == 1 for x in D):
            stats["count"] += 1
            return
        x = min((len(D[i]), i) for i in range(inst.n) if len(D[i]) >= 2)[1]
        a = min(D[x])
        doms = [{a}, D[x] - {a}] if two_way else [{v} for v in sorted(D[x])]
        for dx in doms:
            child = [set(s) for s in D]
            child[x] = dx
            stats["nodes"] += 1
            r = _def_fixpoint(inst, child)
            if r is None:
                stats["fails"] += 1
                continue
            rec(r)

    if any(not s for s in D0):
        stats["fails"] = 1
        return stats
    r = _def_fixpoint(inst, D0)
    if r is None:
        stats["fails"] = 1
        return stats
    rec(r)
    return stats


def test_node_counts_match_independent_search():
    for idx in range(60):
        inst = cspgen.mixed(idx + 500, n=5, dmax=5, m=6)
        s = _def_search(inst)
        r = oracle.solve(inst, oracle.MODE_COUNT)
        assert (r.count, r.nodes, r.fails) == (s["count"], s["nodes"], s["fails"]), idx
    for n in range(4, 8):
        inst = cspgen.queens(n)
        s = _def_search(inst)
        r = oracle.solve(inst, oracle.MODE_COUNT)
        assert (r.count, r.nodes, r.fails) == (s["count"], s["nodes"], s["fails"]), n


def test_queens_node_counts_known():
    # combined pair constraint per column pair: nodes for n = 4..8
    want = {4: 5, 5: 16, 6: 31, 7: 112, 8: 409}
    for n, nodes in want.items():
        assert oracle.solve(cspgen.queens(n), oracle.MODE_COUNT).nodes == nodes


# ----------------------------------------------------------- split & limits

def test_split_invariance_rb_small():
    inst = cspgen.rb(3, n=12, d=6, dens_pm=400, tight_pm=300)
    tot = oracle.solve(inst, oracle.MODE_COUNT).count
    parts = 0
    for v in range(6):
        for w in range(6):
            parts += oracle.solve(inst.fix({0: v, 1: w}), oracle.MODE_COUNT).count
    assert parts == tot and tot > 0


def test_limits():
    inst = cspgen.queens(8)
    r = oracle.solve(inst, oracle.MODE_COUNT, max_nodes=100)
    assert r.verdict == "LIMIT" and r.nodes == 100
    r = oracle.solve(inst, oracle.MODE_COUNT, cap=10)
    assert r.verdict == "LIMIT" and r.count == 10
    r = oracle.solve(inst, oracle.MODE_ALL, sol_cap=5)
    assert r.count == 92 and r.n_written == 5 and r.truncated


def test_malformed_rejected():
    bad = _custom(2, [0, 0], [3, 3], [(2, (0, 0), (0,), ())])
    with pytest.raises(ValueError):
        oracle.solve(bad)
    bad = _custom(2, [0, 0], [3, 3], [(6, (0, 1), (3, 1, 0), ())])
    with pytest.raises(ValueError):
        oracle.solve(bad)


# ------------------------------------------------------ global-constraint twin

@pytest.mark.parametrize("idx", range(3))
def test_global_twin_vs_brute(idx):
    """Scaled twin of the all-different + linear family: exhaustive count."""
    inst = cspgen.global_twin(idx)
    cnt, _ = oracle.brute(inst, limit=10 ** 8)
    r = oracle.solve(inst, oracle.MODE_COUNT)
    assert r.count == cnt and cnt > 0


def test_rb_slices_partition_the_tree():
    """Counting an instance whose root fixpoint keeps every value, in the
    slices x0 = v, reproduces its count and its node count minus the root
    (first-fail branches on x0 first when all domains are equal)."""
    inst = cspgen.rb(7, n=14, d=6, dens_pm=350, tight_pm=300)
    failed, bits, _ = oracle.root(inst)
    assert not failed and all(int(b[0]) == 0b111111 for b in bits)
    full = oracle.solve(inst, oracle.MODE_COUNT)
    parts = [oracle.solve(inst.fix({0: v}), oracle.MODE_COUNT) for v in range(6)]
    assert sum(p.count for p in parts) == full.count
    assert sum(p.nodes for p in parts) == full.nodes - 1
    assert sum(p.fails for p in parts) == full.fails


# ------------------------------------------------- all-different, GAC kind

def test_gac_alldiff_root_is_projection():
    """One all-different of the generalized-arc-consistency kind over random
    initial domains: the root fixpoint keeps exactly the values that occur in
    some assignment of pairwise different values (enumerated)."""
    rng = np.random.default_rng(7)
    seen_prune = 0
    for trial in range(150):
        k = int(rng.integers(2, 6))
        d = int(rng.integers(k - 1, 7))
        lo = [int(v) for v in rng.integers(-2, 3, k)]
        inst = _custom(k, lo, [d] * k, [(7, tuple(range(k)), (), ())])
        init = np.zeros((k, 1), np.uint32)
        for i in range(k):
            bits = rng.integers(0, 2, d)
            if bits.sum() == 0:
                bits[rng.integers(0, d)] = 1
            init[i, 0] = int(sum(int(b) << a for a, b in enumerate(bits)))
        sub = inst.with_init(init)
        doms = [[lo[i] + a for a in range(d) if (int(init[i, 0]) >> a) & 1] for i in range(k)]
        proj = [set() for _ in range(k)]
        for tup in itertools.product(*doms):
            if len(set(tup)) == k:
                for q, v in enumerate(tup):
                    proj[q].add(v)
        failed, bits, _ = oracle.root(sub)
        if not proj[0]:
            assert failed
            continue
        assert not failed
        got = _bits_to_values(sub, bits)
        assert got == [sorted(p) for p in proj], trial
        seen_prune += any(len(proj[q]) < len(doms[q]) for q in range(k))
    assert seen_prune > 20


def test_gac_alldiff_prunes_what_singletons_miss():
    # x0, x1 in {1, 2}, x2 in {1, 2, 3}: the pair x0, x1 takes both 1 and 2,
    # so GAC leaves x2 = 3 at the root; singleton elimination keeps all three
    inst = _custom(3, [1, 1, 1], [3, 3, 3], [(7, (0, 1, 2), (), ())])
    sub = inst.with_init(np.array([[0b011], [0b011], [0b111]], np.uint32))
    failed, bits, _ = oracle.root(sub)
    assert not failed and _bits_to_values(sub, bits) == [[1, 2], [1, 2], [3]]
    weak = sub.with_init(sub.init)
    weak.type = np.array([5], np.int32)
    failed, bits, _ = oracle.root(weak)
    assert not failed and _bits_to_values(weak, bits) == [[1, 2], [1, 2], [1, 2, 3]]


def test_gac_alldiff_counts_and_nodes():
    """Same solutions as the singleton/pigeonhole all-different, never more
    nodes; node counts equal an independent search over the enumerated GAC."""
    fewer = 0
    for idx in range(40):
        inst = cspgen.mixed(idx + 900, n=5, dmax=5, m=5, type_mask=(1 << 5) | (1 << 1) | (1 << 2))
        gac = inst.with_gac()
        a = oracle.solve(inst, oracle.MODE_COUNT)
        b = oracle.solve(gac, oracle.MODE_COUNT)
        assert a.count == b.count and b.nodes <= a.nodes, idx
        fewer += b.nodes < a.nodes
        s = _def_search(gac)
        assert (b.count, b.nodes, b.fails) == (s["count"], s["nodes"], s["fails"]), idx
    for k, s_ in ((3, 3), (4, 6), (5, 5)):
        inst = _custom(k, [0] * k, [s_] * k, [(7, tuple(range(k)), (), ())])
        r = oracle.solve(inst, oracle.MODE_COUNT)
        assert r.count == math.factorial(s_) // math.factorial(s_ - k) and r.fails == 0
    g = cspgen.global_twin(1)
    assert oracle.solve(g.with_gac(), oracle.MODE_COUNT).count == oracle.solve(g, oracle.MODE_COUNT).count
    assert fewer > 0


def test_two_way_branching_counts_and_nodes():
    """2-way branching: the same solutions, node counts equal to the
    independent 2-way search."""
    for idx in range(50):
        inst = cspgen.mixed(idx + 1300, n=5, dmax=5, m=6)
        a = oracle.solve(inst, oracle.MODE_COUNT)
        b = oracle.solve(inst, oracle.MODE_COUNT, two_way=True)
        assert a.count == b.count, idx
        s = _def_search(inst, two_way=True)
        assert (b.count, b.nodes, b.fails) == (s["count"], s["nodes"], s["fails"]), idx
    for n in range(4, 8):
        inst = cspgen.queens(n)
        b = oracle.solve(inst, oracle.MODE_COUNT, two_way=True)
        s = _def_search(inst, two_way=True)
        assert (b.count, b.nodes, b.fails) == (s["count"], s["nodes"], s["fails"]), n


# ------------------------------------------- linear <= with all-different

@pytest.mark.parametrize("n,d", [(3, 5), (4, 6), (5, 5), (6, 9)])
def test_linear_ad_root_fails_below_the_distinct_minimum(n, d):
    """n variables over 0..d-1, all different, sum x_i <= b: pairwise
    different values sum to at least 0 + 1 + ... + (n-1) = n(n-1)/2.  With
    b one below it the all-different-aware propagator fails at the root (1
    node, 1 failure) while the plain bound (0) has to search; with b equal
    to it the solutions are the n! orderings of 0..n-1."""
    lo_sum = n * (n - 1) // 2
    for b in (lo_sum - 1, lo_sum):
        cons = [(5, tuple(range(n)), (), ()), (6, tuple(range(n)), (b,) + (1,) * n, ())]
        plain = _custom(n, [0] * n, [d] * n, cons)
        ad = _custom(n, [0] * n, [d] * n, [cons[0], (8, tuple(range(n)), (b,) + (1,) * n, ())])
        rp = oracle.solve(plain, oracle.MODE_COUNT)
        ra = oracle.solve(ad, oracle.MODE_COUNT)
        assert ra.count == rp.count
        if b < lo_sum:
            assert ra.count == 0 and (ra.nodes, ra.fails) == (1, 1)
            assert rp.nodes > 1
        else:
            assert ra.count == math.factorial(n)
            assert ra.nodes <= rp.nodes


def test_linear_ad_weighted_minimum():
    """Coefficients (3, 2, 1) over 0..4, all different: the smallest weighted
    sum of three different values puts the largest coefficient on the
    smallest value, 3*0 + 2*1 + 1*2 = 4 (rearrangement).  b = 3 fails at the
    root; b = 4 has exactly the solution (0, 1, 2)."""
    for b, want in ((3, 0), (4, 1)):
        inst = _custom(3, [0] * 3, [5] * 3, [(5, (0, 1, 2), (), ()), (8, (0, 1, 2), (b, 3, 2, 1), ())])
        r = oracle.solve(inst, oracle.MODE_ALL, sol_cap=10)
        assert r.count == want
        if want == 0:
            assert (r.nodes, r.fails) == (1, 1)
        else:
            assert r.solutions.tolist() == [[0, 1, 2]]


@pytest.mark.parametrize("idx", range(6))
def test_linear_ad_counts_match_brute_force(idx):
    """The global family's twins with the all-different-aware linear
    propagator: the same solution counts as brute force and as the plain
    linear propagator, every solution verified, and root domains inside the
    plain propagator's.  (Node counts may go either way: first-fail picks
    its variables from different domain sizes.)"""
    g = cspgen.global_twin(idx)
    ad = g.with_linear_ad()
    bf = oracle.brute(g, limit=10 ** 8)
    assert bf is not None
    rp = oracle.solve(g, oracle.MODE_COUNT)
    ra = oracle.solve(ad, oracle.MODE_COUNT)
    assert ra.count == rp.count == bf[0]
    ref = oracle.solve(ad, oracle.MODE_ALL, sol_cap=bf[0] + 1)
    assert ref.n_written == bf[0]
    for row in ref.solutions:
        assert oracle.verify(g, row)
    fp, bp, _ = oracle.root(g)
    fa, ba, _ = oracle.root(ad)
    assert fa or not fp
    if not fa:
        assert np.all((ba & ~bp) == 0)


@pytest.mark.parametrize("idx", range(12))
def test_linear_ad_node_counts_match_independent_search(idx):
    """Small twins (5 variables over 0..4, all-different over 3) searched by
    the independent definition-level search, whose group bound enumerates
    every assignment of pairwise different values: equal counts, nodes and
    failures."""
    ad = cspgen.global_twin(idx, n=5, d=5, k_ad=3).with_linear_ad()
    s = _def_search(ad)
    r = oracle.solve(ad, oracle.MODE_COUNT)
    assert (r.count, r.nodes, r.fails) == (s["count"], s["nodes"], s["fails"]), idx
