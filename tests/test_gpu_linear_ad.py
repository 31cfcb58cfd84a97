"""GPU parity of the linear <= propagated together with the all-different
groups inside its scope (constraint type 8) against the oracle: root
fixpoints on random small instances (shifted value ranges, domains of one to
eight words, one or two groups of either all-different type, ungrouped
variables), counts, nodes and failures on the global family's twins (single
and batched), the closed-form root failure, and the full-size global
instance with verified answers."""
import math
import sys

import numpy as np
import pytest

import cspgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cb():
    from paper_1909_09213_amd import cubics
    return cubics


@pytest.fixture(scope="module")
def ctx(cb):
    c = cb.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def _instance(lo, d, cons, init=None):
    """cons: (type, scope, params)."""
    n = len(lo)
    var_off, vars_, par_off, params = [0], [], [0], []
    for _, sc, par in cons:
        vars_ += list(sc)
        var_off.append(len(vars_))
        params += list(par)
        par_off.append(len(params))
    inst = cspgen.Instance(
        lo=np.array(lo, np.int32), dsize=np.array(d, np.int32),
        type=np.array([c[0] for c in cons], np.int32),
        arity=np.array([len(c[1]) for c in cons], np.int32),
        var_off=np.array(var_off, np.int64), vars=np.array(vars_, np.int32),
        par_off=np.array(par_off, np.int64), params=np.array(params, np.int64),
        tab_off=np.zeros(len(cons) + 1, np.int64), tabs=np.zeros(0, np.uint32))
    return inst.with_init(init) if init is not None else inst


def _random_case(rng, dmax):
    n = int(rng.integers(3, 13))
    d = [int(rng.integers(max(2, dmax // 2), dmax + 1)) for _ in range(n)]
    # shifted value ranges in a quarter of the cases, else shared ones
    lo = [int(v) for v in rng.integers(-3, 4, n)] if rng.random() < 0.25 else [0] * n
    W = (max(d) + 31) // 32
    init = np.zeros((n, W), np.uint32)
    for i in range(n):
        # mostly low values, so that group members share their minima
        win = min(d[i], int(rng.integers(n // 2 + 2, n + 4)))
        for a in rng.choice(win, size=int(rng.integers(1, win + 1)), replace=False):
            init[i, a // 32] |= np.uint32(1 << (int(a) % 32))
        if rng.random() < 0.5:
            a = int(rng.integers(0, d[i]))
            init[i, a // 32] |= np.uint32(1 << (a % 32))
    perm = [int(v) for v in rng.permutation(n)]
    k1 = int(rng.integers(2, max(3, (2 * n) // 3) + 1))
    cons = [(int(rng.choice([cspgen.ALLDIFF, cspgen.ALLDIFF_GAC])), perm[:k1], ())]
    if n - k1 >= 3 and rng.random() < 0.6:
        k2 = int(rng.integers(2, n - k1))
        cons.append((int(rng.choice([cspgen.ALLDIFF, cspgen.ALLDIFF_GAC])), perm[k1:k1 + k2], ()))
    scope = [int(v) for v in rng.permutation(n)][: int(rng.integers(max(3, n - 2), n + 1))]
    need = set(v for c in cons for v in c[1])
    scope += [v for v in need if v not in scope]
    coef = [int(v) for v in rng.integers(1, 10, len(scope))]
    # vals: the init bits' values
    mins = [lo[v] + min(a for a in range(d[v]) if (int(init[v, a // 32]) >> (a % 32)) & 1) for v in scope]
    maxs = [lo[v] + max(a for a in range(d[v]) if (int(init[v, a // 32]) >> (a % 32)) & 1) for v in scope]
    smin = sum(c * m for c, m in zip(coef, mins))
    smax = sum(c * m for c, m in zip(coef, maxs))
    r = rng.random()
    b = (smin - 1 if r < 0.05 else int(rng.integers(smin, smin + 3 * max(coef) + 1)) if r < 0.8
         else int(rng.integers(smin, max(smin, smax) + 1)))
    cons.append((cspgen.LINEAR_LE_AD, scope, [b] + coef))
    return _instance(lo, d, cons, init)


@pytest.mark.parametrize("dmax", [6, 40, 100, 250])
@pytest.mark.parametrize("layout", [1, 2])
def test_linear_ad_root_fixpoints(ctx, cb, dmax, layout):
    rng = np.random.default_rng(7000 + dmax)
    for trial in range(60):
        inst = _random_case(rng, dmax)
        _say("linear_ad root", dmax, layout, trial, inst.n)
        failed, bits = ctx.root(ctx.load(inst), layout)
        rf, rbits, _ = oracle.root(inst)
        assert failed == rf, trial
        if not rf:
            assert np.array_equal(bits, rbits), trial


@pytest.mark.parametrize("idx", range(6))
def test_linear_ad_global_twins(ctx, cb, idx):
    inst = cspgen.global_twin(idx).with_linear_ad()
    _say("linear_ad twin", idx)
    ref = oracle.solve(inst, oracle.MODE_COUNT)
    prob = ctx.load(inst)
    for split in (0, 4096):
        r = ctx.solve(prob, cb.MODE_COUNT, split_target=split)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), split


def test_linear_ad_all_solutions_and_batch(ctx, cb):
    inst = cspgen.global_twin(1, n=7, d=8, k_ad=4).with_linear_ad()
    ref = oracle.solve(inst, oracle.MODE_ALL, sol_cap=200000)
    r = ctx.solve(ctx.load(inst), cb.MODE_ALL, sol_capacity=ref.count)
    assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails)
    assert sorted(map(tuple, r.solutions.tolist())) == sorted(map(tuple, ref.solutions.tolist()))
    insts = [cspgen.global_twin(i, n=7, d=7, k_ad=4).with_linear_ad() for i in range(32)]
    res = ctx.solve_batch([ctx.load(x) for x in insts], cb.MODE_COUNT)
    for i, (x, got) in enumerate(zip(insts, res)):
        want = oracle.solve(x, oracle.MODE_COUNT)
        assert (got.count, got.nodes, got.fails) == (want.count, want.nodes, want.fails), i


@pytest.mark.parametrize("n", [4, 6, 9])
def test_linear_ad_closed_form_root_failure(ctx, cb, n):
    """All different over 0..d-1 with sum <= n(n-1)/2 - 1 fails at the root;
    at n(n-1)/2 the solutions are the n! orders of 0..n-1."""
    lo_sum = n * (n - 1) // 2
    for b, want in ((lo_sum - 1, 0), (lo_sum, math.factorial(n))):
        inst = _instance([0] * n, [n + 3] * n, [(cspgen.ALLDIFF, list(range(n)), ()),
                                                (cspgen.LINEAR_LE_AD, list(range(n)), [b] + [1] * n)])
        r = ctx.solve(ctx.load(inst), cb.MODE_COUNT)
        assert r.count == want
        if want == 0:
            assert (r.nodes, r.fails) == (1, 1)


def test_linear_ad_full_size_capped(ctx, cb):
    inst = cspgen.global_family(0).with_linear_ad()
    _say("global full size with linear_ad, cap 1e5")
    r = ctx.solve(ctx.load(inst), cb.MODE_COUNT, max_solutions=10 ** 5, split_target=65536,
                  sol_capacity=500)
    assert r.verdict == "LIMIT" and r.count == 10 ** 5
    assert len({tuple(x) for x in r.solutions.tolist()}) == 500
    for row in r.solutions:
        assert oracle.verify(inst, row)


def test_linear_ad_rejects_a_repeated_variable(ctx, cb):
    inst = _instance([0] * 3, [4] * 3, [(cspgen.ALLDIFF, [0, 1], ()),
                                        (cspgen.LINEAR_LE_AD, [0, 1, 0], [5, 1, 1, 1])])
    with pytest.raises(cb.CubicsError):
        ctx.load(inst)
