"""Large-neighbourhood search (minimise sum c_i x_i over the solutions)
against the optimum enumerated with the oracle's brute force."""
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


def _optimum(inst, obj, limit=10 ** 8):
    cnt, sols = oracle.brute(inst, limit=limit, sol_cap=400000)
    assert cnt <= 400000
    if cnt == 0:
        return None
    return int((sols.astype(np.int64) @ np.asarray(obj, np.int64)).min())


def test_lns_reaches_and_proves_the_optimum_on_small_instances(ctx, cb):
    rng = np.random.default_rng(4)
    solved = 0
    for idx in range(24):
        inst = cspgen.mixed(idx + 8800, n=6, dmax=7, m=6)
        obj = rng.integers(0, 6, inst.n)
        obj[rng.integers(0, inst.n)] += 1
        opt = _optimum(inst, obj)
        _say("lns small", idx, opt)
        r = ctx.lns(inst, obj, neighborhoods=16, max_nodes=0, seed=idx)
        if opt is None:
            assert not r["found"]
            continue
        solved += 1
        assert r["found"] and r["optimal"] and r["objective"] == opt, idx
        assert oracle.verify(inst, r["best"]) and int(np.dot(r["best"], obj)) == opt
    assert solved >= 10


def test_lns_on_the_global_twin(ctx, cb):
    inst = cspgen.global_twin(0)
    obj = np.arange(1, inst.n + 1)
    opt = _optimum(inst, obj)
    r = ctx.lns(inst, obj, neighborhoods=128, relax_pm=400, max_nodes=0, seed=3)
    _say("twin", opt, r)
    assert r["optimal"] and r["objective"] == opt
    assert oracle.verify(inst, r["best"])


def test_lns_improves_with_neighbourhoods_under_a_budget(ctx, cb):
    """RB n=30 d=10: copy 0 cannot finish within its budget, so only the
    neighbourhoods improve the first solution; every incumbent verifies."""
    inst = cspgen.rb(3, n=30, d=10, dens_pm=250, tight_pm=300)
    obj = np.ones(inst.n, np.int64)
    r = ctx.lns(inst, obj, neighborhoods=512, relax_pm=250, max_nodes=20000, rounds=6, seed=9)
    _say("rb lns", r["objective"], r["improvements"], r["rounds"], r["nodes"])
    assert r["found"] and r["improvements"] >= 1
    assert oracle.verify(inst, r["best"]) and int(r["best"].sum()) == r["objective"]


def test_lns_errors(ctx, cb):
    inst = cspgen.queens(5)
    with pytest.raises(Exception):
        ctx.lns(inst, -np.ones(5, np.int64))
    with pytest.raises(Exception):
        ctx.lns(inst, np.zeros(5, np.int64))
    r = ctx.lns(cspgen.queens(3), np.ones(3, np.int64), neighborhoods=4)
    assert not r["found"]
