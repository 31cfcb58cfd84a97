"""Write the stored expected values of the large parity tests.

Every value here comes from the CPU oracle (``oracle/``) run on the seeded
generators (``cspgen/``); nothing is read from the GPU library.  Runs on the
CPU with one process per core:

    python tests/golden/make_goldens.py sweep     # sweep_verdicts.txt
    python tests/golden/make_goldens.py rb_slice  # rb_slice_x0_1.txt
    python tests/golden/make_goldens.py rb_tight  # rb_tight400.txt
    python tests/golden/make_goldens.py rb_depth2 # rb_depth2.txt

sweep: the 4096 instances of the batched find-first configuration (base
seed 3, indices 0..4095), each solved by the oracle in find-first mode with
a node budget (verdict SAT / UNSAT / LIMIT, nodes, fails).  An UNSAT verdict
explores the whole first-fail tree, so its node and failure counts are those
any solver with the same propagation and branching reaches.

rb_slice: the RB instance of the count configuration (n=40, d=16, density
0.25, tightness 0.35, seed 2 index 0) restricted to x0 = 1, counted as the
16 sub-CSPs x1 = v (a partition of its solutions).

rb_tight: the same generator at tightness 0.40 (t = 102 forbidden pairs per
table), counted exhaustively (count, nodes, fails).

rb_depth2: seeded sub-CSPs of the count instance with x0 and x1 fixed,
counted exhaustively (count, nodes, fails).
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SWEEP_BUDGET = 20_000
SWEEP_FILE = os.path.join(HERE, "sweep_verdicts.txt")
RB_SLICE_FILE = os.path.join(HERE, "rb_slice_x0_1.txt")
RB_TIGHT_FILE = os.path.join(HERE, "rb_tight400.txt")
RB_DEPTH2_FILE = os.path.join(HERE, "rb_depth2.txt")
RB_DEPTH2_PAIRS = 6
BATCH = 4096


def _procs() -> int:
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def _sweep_one(i):
    import cspgen
    import oracle
    inst = cspgen.rb_sweep(i)
    r = oracle.solve(inst, oracle.MODE_FIRST, max_nodes=SWEEP_BUDGET)
    return i, r.verdict, r.nodes, r.fails


def sweep():
    t0 = time.time()
    # hard instances first, so that the pool's tail is short: order by size
    import cspgen
    order = sorted(range(BATCH), key=lambda i: -cspgen.rb_sweep(i).m)
    rows = {}
    with mp.Pool(_procs()) as pool:
        for k, (i, v, nodes, fails) in enumerate(pool.imap_unordered(_sweep_one, order, chunksize=1)):
            rows[i] = (v, nodes, fails)
            if k % 256 == 0:
                print(f"sweep {k}/{BATCH} {time.time() - t0:.0f}s", flush=True)
    with open(SWEEP_FILE, "w") as f:
        f.write("# Oracle find-first verdicts of the batched sweep configuration: 4096\n"
                "# random binary CSPs, base seed 3, indices 0..4095 (n U{20..120},\n"
                "# d U{8..64}, density 100..300 per mille, tightness 200..500 per mille),\n"
                f"# node budget {SWEEP_BUDGET} per instance (LIMIT = unresolved within it).\n"
                "# Written by tests/golden/make_goldens.py sweep (oracle only).\n"
                f"# budget {SWEEP_BUDGET}\n"
                "# index verdict nodes fails\n")
        for i in range(BATCH):
            v, nodes, fails = rows[i]
            f.write(f"{i} {v} {nodes} {fails}\n")
    print(f"wrote {SWEEP_FILE} in {time.time() - t0:.0f}s", flush=True)


def _rb_count(args):
    import cspgen
    import oracle
    kind, fix, tight = args
    inst = cspgen.rb(0, n=40, d=16, dens_pm=250, tight_pm=tight, base=cspgen.SEED_RB)
    if fix:
        inst = inst.fix(dict(fix))
    t = time.time()
    r = oracle.solve(inst, oracle.MODE_COUNT)
    assert r.verdict in ("SAT", "UNSAT")
    return kind, fix, r.count, r.nodes, r.fails, time.time() - t


def rb_slice():
    jobs = [("slice", ((0, 1), (1, v)), 350) for v in range(16)]
    with mp.Pool(_procs()) as pool:
        out = pool.map(_rb_count, jobs, chunksize=1)
    with open(RB_SLICE_FILE, "w") as f:
        f.write("# RB n=40 d=16 density 250 tightness 350 per mille (seed 2 index 0),\n"
                "# sub-CSPs x0 = 1, x1 = v (v = 0..15), counted exhaustively by the oracle.\n"
                "# Their counts partition the solutions of the slice x0 = 1.\n"
                "# Written by tests/golden/make_goldens.py rb_slice (oracle only).\n"
                "# x1 count nodes fails\n")
        for _, fix, count, nodes, fails, _ in out:
            f.write(f"{fix[1][1]} {count} {nodes} {fails}\n")
        f.write(f"# total {sum(o[2] for o in out)}\n")
    print(f"wrote {RB_SLICE_FILE}", flush=True)


def rb_tight():
    kind, fix, count, nodes, fails, dt = _rb_count(("tight", (), 400))
    with open(RB_TIGHT_FILE, "w") as f:
        f.write("# RB n=40 d=16 density 250 tightness 400 per mille (t = 102 of 256 pairs\n"
                "# forbidden per table; seed 2 index 0), counted exhaustively by the oracle.\n"
                "# Written by tests/golden/make_goldens.py rb_tight (oracle only).\n"
                f"count {count}\nnodes {nodes}\nfails {fails}\n")
    print(f"wrote {RB_TIGHT_FILE} ({dt:.0f}s)", flush=True)


def rb_depth2():
    import numpy as np
    rng = np.random.default_rng(22)
    pairs = [tuple(int(x) for x in rng.integers(0, 16, 2)) for _ in range(RB_DEPTH2_PAIRS)]
    jobs = [("d2", ((0, a), (1, b)), 350) for a, b in pairs]
    with mp.Pool(_procs()) as pool:
        out = pool.map(_rb_count, jobs, chunksize=1)
    with open(RB_DEPTH2_FILE, "w") as f:
        f.write("# RB n=40 d=16 density 250 tightness 350 per mille (seed 2 index 0),\n"
                "# seeded sub-CSPs with x0 = a and x1 = b fixed (numpy default_rng(22)),\n"
                "# counted exhaustively by the oracle.\n"
                "# Written by tests/golden/make_goldens.py rb_depth2 (oracle only).\n"
                "# a b count nodes fails\n")
        for _, fix, count, nodes, fails, _ in out:
            f.write(f"{fix[0][1]} {fix[1][1]} {count} {nodes} {fails}\n")
    print(f"wrote {RB_DEPTH2_FILE}", flush=True)


if __name__ == "__main__":
    what = sys.argv[1:] or ["sweep", "rb_slice", "rb_tight", "rb_depth2"]
    for w in what:
        {"sweep": sweep, "rb_slice": rb_slice, "rb_tight": rb_tight, "rb_depth2": rb_depth2}[w]()
