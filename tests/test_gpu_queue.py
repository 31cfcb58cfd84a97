"""The work queue at full occupancy and under a stop.

A search of ~10^6 nodes on thousands of waves keeps most of them idle: they
hold tickets or wait on their workgroup's token while a few busy waves donate
frames.  The node and failure counts of a d-way first-fail search are fixed
by the tree, so they must match the oracle's exactly however the work was
split.  A time limit must stop a long search, drain the tasks still queued
and end the launch promptly, in every layout."""
import sys

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


# RB n=30 d=10, density 0.25, tightness 0.39: 1.1e6 nodes (oracle ~1.5 s)
STRESS = dict(index=0, n=30, d=10, dens_pm=250, tight_pm=390)


@pytest.fixture(scope="module")
def stress_ref():
    inst = cspgen.rb(**STRESS)
    return inst, oracle.solve(inst, oracle.MODE_COUNT)


@pytest.mark.parametrize("layout", [1, 3])  # LANE, VAR
@pytest.mark.parametrize("workers", [0, 64])  # every co-resident wave; a few
def test_full_occupancy_counts(ctx, cb, stress_ref, layout, workers):
    inst, ref = stress_ref
    assert ref.verdict == "SAT" and ref.nodes > 10 ** 6
    _say("queue stress", STRESS, "layout", layout, "workers", workers)
    p = ctx.load(inst)
    for rep in range(2):  # the second launch reuses the queue and trail buffers
        r = ctx.solve(p, cb.MODE_COUNT, layout=layout, workers=workers)
        assert (r.count, r.nodes, r.fails) == (ref.count, ref.nodes, ref.fails), rep
        assert r.tasks >= 1
    p.free()


@pytest.mark.parametrize("layout", [1, 2, 3])
def test_time_limit_stops_and_drains(ctx, cb, layout):
    # a slice of the RB n=40 d=16 instance: 1.3e10 nodes, seconds of search
    inst = cspgen.rb(0, n=40, d=16, dens_pm=250, tight_pm=350, base=cspgen.SEED_RB).fix({0: 1})
    _say("time limit, layout", layout)
    p = ctx.load(inst)
    r = ctx.solve(p, cb.MODE_COUNT, layout=layout, time_ms=200)
    assert r.verdict == "LIMIT"
    assert 0 < r.nodes < 13383873410
    # the stop is seen within 2048 nodes of every worker; the queued tasks
    # are then claimed and skipped
    assert r.kernel_ms < 1200, r.kernel_ms
    # the context stays usable: a complete small search right after
    q = ctx.load(cspgen.queens(8))
    assert ctx.solve(q, cb.MODE_COUNT, layout=layout).count == 92
    q.free()
    p.free()
