"""GPU parity at domain widths of 2, 4 and 8 words per domain (33..256
values): the search kernels compiled for those widths against the CPU oracle
on instances it finishes in well under a second.

For every instance: the root fixpoint bit for bit; count, node and failure
counts in count mode under d-way and 2-way branching, with the default
worker count (donation), one worker, and an eager split; the sorted solution
set in all mode; a verified assignment and the verdict in first mode.  The
table instances run in the LANE layout and, where domains have at most 64
values, in the SEG layout; the all-different + linear instances (the global
family at its full domain width, 0..255) run in the LANE layout, which is the
only one that carries global constraints, with the all-different propagated
both ways (singleton elimination + pigeonhole, and generalized arc
consistency)."""
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


def _canon(rows):
    return sorted(tuple(int(v) for v in r) for r in rows)


def _global(i, gac=False):
    inst = cspgen.global_family(i, n=5, lo=0, d=256, n_ad=1, k_ad=4, n_lin=2, lin_k=0, amax=9,
                                b_pm=15, base=cspgen.SEED_GLOBAL + 200)
    return inst.with_gac() if gac else inst


# (name, generator, device words per domain: the kernel width it exercises)
FAMILIES = [
    ("rb_n9_d40", lambda i: cspgen.rb(i, n=9, d=40, dens_pm=600, tight_pm=700), 2),
    ("rb_n8_d60", lambda i: cspgen.rb(i, n=8, d=60, dens_pm=700, tight_pm=750), 2),
    ("sweep_w2", lambda i: cspgen.rb_sweep(i, base=cspgen.SEED_SWEEP + 300, nlo=7, nhi=10,
                                           dlo=33, dhi=64, plo=500, phi=800, tlo=620, thi=800), 2),
    ("rb_n6_d90", lambda i: cspgen.rb(i, n=6, d=90, dens_pm=900, tight_pm=800), 3),
    ("rb_n5_d128", lambda i: cspgen.rb(i, n=5, d=128, dens_pm=1000, tight_pm=820), 4),
    ("rb_n5_d200", lambda i: cspgen.rb(i, n=5, d=200, dens_pm=1000, tight_pm=880), 7),
    ("global_d256", lambda i: _global(i), 8),
    ("global_gac_d256", lambda i: _global(i, gac=True), 8),
]
CASES = [(name, gen, w, i) for name, gen, w in FAMILIES for i in range(2)]


def _layouts(inst):
    return [1, 2] if inst.dmax <= 64 and inst.name.startswith(("rb", "sweep")) else [1]


@pytest.mark.parametrize("name,gen,words,idx", CASES, ids=[f"{c[0]}-{c[3]}" for c in CASES])
def test_wide_exact(ctx, cb, name, gen, words, idx):
    inst = gen(idx)
    prob = ctx.load(inst)
    assert prob.W == words, (name, prob.W)
    rf, rbits, _ = oracle.root(inst)
    ref = {tw: oracle.solve(inst, oracle.MODE_COUNT, two_way=tw) for tw in (False, True)}
    assert ref[False].count == ref[True].count
    for layout in _layouts(inst):
        _say(name, idx, "layout", layout)
        failed, bits = ctx.root(prob, layout)
        assert failed == rf, (name, idx, layout)
        if not rf:
            assert np.array_equal(bits, rbits), (name, idx, layout)
        for tw in (False, True):
            want = (ref[tw].count, ref[tw].nodes, ref[tw].fails)
            for kw in ({}, {"workers": 1}, {"split_target": 64}):
                r = ctx.solve(prob, cb.MODE_COUNT, layout=layout, two_way=tw, **kw)
                assert (r.count, r.nodes, r.fails) == want, (name, idx, layout, tw, kw)
        f = ctx.solve(prob, cb.MODE_FIRST, layout=layout)
        assert f.verdict == ("SAT" if ref[False].count else "UNSAT"), (name, idx, layout)
        if f.verdict == "SAT":
            assert oracle.verify(inst, f.solutions[0]), (name, idx, layout)


@pytest.mark.parametrize("name,gen,words", FAMILIES, ids=[f[0] for f in FAMILIES])
def test_wide_solution_sets(ctx, cb, name, gen, words):
    inst = gen(0)
    ref = oracle.solve(inst, oracle.MODE_ALL, sol_cap=20000)
    assert 0 < ref.count <= 20000, (name, ref.count)
    prob = ctx.load(inst)
    for layout in _layouts(inst):
        r = ctx.solve(prob, cb.MODE_ALL, layout=layout, sol_capacity=ref.count)
        assert r.count == ref.count and not r.truncated, (name, layout)
        assert _canon(r.solutions) == _canon(ref.solutions), (name, layout)


def test_wide_batch_mixed_widths(ctx, cb):
    """One launch over instances of every width (the batch runs at the
    widest): per-instance counts, nodes and failures equal the oracle's."""
    insts = [gen(i) for _, gen, _ in FAMILIES for i in range(2)]
    probs = [ctx.load(x) for x in insts]
    res = ctx.solve_batch(probs, cb.MODE_COUNT)
    for inst, r in zip(insts, res):
        ref = oracle.solve(inst, oracle.MODE_COUNT)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), inst.name
