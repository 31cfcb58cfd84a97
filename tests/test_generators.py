"""The seeded generators both sides share: SplitMix64 as published, unbiased
bounded draws, deterministic instances, and the instance shapes the
configurations name."""
import numpy as np

import cspgen

M64 = (1 << 64) - 1


def _splitmix64(state, count):
    # Steele, Lea and Flood (OOPSLA 2014): state += golden gamma, then the
    # variant-13 finalizer
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


def test_splitmix64_stream():
    for seed in (0, 1, 12345, 0xDEADBEEF, (1 << 63) + 5):
        assert [int(v) for v in cspgen.rng_stream(seed, 16)] == _splitmix64(seed, 16)
    # the widely quoted first output for state 0
    assert int(cspgen.rng_stream(0, 1)[0]) == 0xE220A8397B1DCDAF


def test_bounded_draws_in_range_and_unbiased():
    for r in (1, 2, 3, 7, 10, 1000):
        v = cspgen.rng_below(99, r, 20000).astype(np.int64)
        assert v.min() >= 0 and v.max() < r
        if r > 1:
            counts = np.bincount(v, minlength=r)
            exp = 20000 / r
            assert np.all(np.abs(counts - exp) < 6 * np.sqrt(exp))


def test_instance_seed_and_determinism():
    assert cspgen.instance_seed(3, 5) == 3 ^ ((5 * 0x9E3779B97F4A7C15) & M64)
    a, b = cspgen.rb_sweep(17), cspgen.rb_sweep(17)
    for f in ("lo", "dsize", "type", "arity", "var_off", "vars", "tabs"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = cspgen.rb_sweep(18)
    assert not (np.array_equal(a.vars, c.vars) and np.array_equal(a.tabs, c.tabs))


def test_configuration_shapes():
    rb = cspgen.rb(0)
    assert rb.n == 40 and int(rb.dsize.max()) == 16 and rb.m == 195
    for c in range(rb.m):  # 90 of 256 pairs forbidden in every table
        bits = np.unpackbits(rb.tab(c).view(np.uint8), bitorder="little").reshape(16, 32)[:, :16]
        assert int(bits.sum()) == 256 - 90
    q = cspgen.queens(8)
    assert q.n == 8 and q.m == 28 and int(q.lo[0]) == 1
    g = cspgen.global_family(0)
    types = list(g.type)
    assert g.n == 200 and int(g.dsize.max()) == 256
    assert types.count(cspgen.ALLDIFF) == 10 and types.count(cspgen.LINEAR_LE) == 30
    for i in range(400):
        s = cspgen.rb_sweep(i)
        assert 20 <= s.n <= 120 and 8 <= int(s.dsize[0]) <= 64
