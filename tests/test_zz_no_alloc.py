"""The allocation-free batch entry point, cubics_solve_batch_static, against
cubics_solve_batch on the same inputs: two calls in a row (the second with a
smaller batch, which reuses the static scratch the first left behind), count
mode with exact counts, node and failure counts, find-first mode with
verdicts and verified assignments, domains of one and of eight words, and
the size limit of the static scratch."""
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


def _batch(count):
    insts = [cspgen.rb_sweep(i, base=123, nlo=12, nhi=18, dlo=5, dhi=9, plo=350, phi=550,
                             tlo=300, thi=450) for i in range(count)]
    # eight-word domains: all-different + linear <= over 0..255
    insts += [cspgen.global_family(i, n=5, lo=0, d=256, n_ad=1, k_ad=4, n_lin=2, lin_k=0, amax=9,
                                   b_pm=15, base=cspgen.SEED_GLOBAL + 200) for i in range(2)]
    return insts


def test_static_batch_matches_solve_batch(ctx, cb):
    for count in (40, 6):  # the second call is smaller
        insts = _batch(count)
        probs = [ctx.load(x) for x in insts]
        a = ctx.solve_batch(probs, cb.MODE_COUNT, max_nodes=50_000_000, static_scratch=True)
        b = ctx.solve_batch(probs, cb.MODE_COUNT, max_nodes=50_000_000)
        for inst, ra, rb in zip(insts, a, b):
            assert ra.verdict == rb.verdict != "LIMIT", inst.name
            assert (ra.count, ra.nodes, ra.fails) == (rb.count, rb.nodes, rb.fails), inst.name
            ref = oracle.solve(inst, oracle.MODE_COUNT)
            assert (ra.count, ra.nodes, ra.fails) == (ref.count, ref.nodes, ref.fails), inst.name
        fa = ctx.solve_batch(probs, cb.MODE_FIRST, static_scratch=True)
        fb = ctx.solve_batch(probs, cb.MODE_FIRST)
        for inst, ra, rb in zip(insts, fa, fb):
            assert ra.verdict == rb.verdict, inst.name
            if ra.verdict == "SAT":
                assert oracle.verify(inst, ra.solutions[0]), inst.name


def test_static_batch_rejects_what_needs_allocation(ctx, cb):
    probs = [ctx.load(cspgen.queens(6))]
    with pytest.raises(cb.CubicsError) as e:
        ctx.solve_batch(probs, cb.MODE_COUNT, use_graph=True, static_scratch=True)
    assert e.value.code == -1
    # 256 variables over 0..255 under 2-way branching: one worker's trail
    # (1 + 256 * 255 frames of 2080 words) exceeds the 256 MiB scratch
    n, d = 256, 256
    inst = cspgen.Instance(lo=np.zeros(n, np.int32), dsize=np.full(n, d, np.int32),
                           type=np.zeros(0, np.int32), arity=np.zeros(0, np.int32),
                           var_off=np.zeros(1, np.int64), vars=np.zeros(0, np.int32),
                           par_off=np.zeros(1, np.int64), params=np.zeros(0, np.int64),
                           tab_off=np.zeros(1, np.int64), tabs=np.zeros(0, np.uint32))
    big = ctx.load(inst)
    with pytest.raises(cb.CubicsError) as e:
        ctx.solve_batch([big], cb.MODE_FIRST, two_way=True, static_scratch=True)
    assert e.value.code == -4
