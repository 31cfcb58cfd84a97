"""Seeded synthetic CSP instances shared by the tests, the CPU oracle runs and
the benchmark.

The generators live in ``gen.c`` (SplitMix64 streams, partial Fisher-Yates
sampling) and hold none of the solving method.  An :class:`Instance` is the
flat constraint list both solvers read: per-variable ``lo``/``dsize`` and a
CSR-style constraint table (``type``, ``arity``, scope, integer parameters,
packed bit rows).  See the header comment of ``gen.c`` for the type codes.

Families (the workloads of the benchmark configurations):

* :func:`queens` - n-queens, one combined pair constraint per column pair.
* :func:`worked_example` - the paper's two-variable example (Sec. 1.1).
* :func:`rb` - random binary CSP with exact density and tightness.
* :func:`rb_sweep` - one instance of the batched sweep (n, d, density and
  tightness drawn per instance).
* :func:`tree` - tree-structured binary CSP.
* :func:`global_family` - all-different + linear <= instances.
* :func:`mixed` - tiny instances mixing all constraint types.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

UNARY, TABLE2, NEQ, LT, QUEENS, ALLDIFF, LINEAR_LE, ALLDIFF_GAC, LINEAR_LE_AD = range(9)
TYPE_NAMES = ["UNARY", "TABLE2", "NEQ", "LT", "QUEENS", "ALLDIFF", "LINEAR_LE", "ALLDIFF_GAC",
              "LINEAR_LE_AD"]

GOLDEN64 = 0x9E3779B97F4A7C15

# base seeds of the configuration families
SEED_RB = 2          # random binary CSP, count all
SEED_SWEEP = 3       # batched find-first sweep
SEED_GLOBAL = 4      # all-different + linear
SEED_TRAIN = 5       # learned-branching training seeds
SEED_EVAL = 6        # learned-branching held-out seeds

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libcspgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libcspgen.so next to it (gcc, -O2)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "gen.c")
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


class _GenInst(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("m", ctypes.c_int32),
        ("lo", ctypes.POINTER(ctypes.c_int32)), ("dsize", ctypes.POINTER(ctypes.c_int32)),
        ("type", ctypes.POINTER(ctypes.c_int32)), ("arity", ctypes.POINTER(ctypes.c_int32)),
        ("var_off", ctypes.POINTER(ctypes.c_int64)), ("vars", ctypes.POINTER(ctypes.c_int32)),
        ("par_off", ctypes.POINTER(ctypes.c_int64)), ("params", ctypes.POINTER(ctypes.c_int64)),
        ("tab_off", ctypes.POINTER(ctypes.c_int64)), ("tabs", ctypes.POINTER(ctypes.c_uint32)),
        ("cap_m", ctypes.c_int64), ("cap_vars", ctypes.c_int64),
        ("cap_par", ctypes.c_int64), ("cap_tab", ctypes.c_int64),
    ]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.POINTER(_GenInst)
        u64, i32 = ctypes.c_uint64, ctypes.c_int
        lib.gen_queens.argtypes = [i32]
        lib.gen_worked_example.argtypes = [i32]
        lib.gen_rb.argtypes = [u64, i32, i32, i32, i32]
        lib.gen_rb_sweep.argtypes = [u64] + [i32] * 8
        lib.gen_tree.argtypes = [u64, i32, i32, i32]
        lib.gen_global.argtypes = [u64] + [i32] * 9
        lib.gen_mixed.argtypes = [u64, i32, i32, i32, i32]
        for f in ("gen_queens", "gen_worked_example", "gen_rb", "gen_rb_sweep",
                  "gen_tree", "gen_global", "gen_mixed"):
            getattr(lib, f).restype = P
        lib.gen_free.argtypes = [P]
        lib.gen_free.restype = None
        lib.gen_instance_seed.argtypes = [u64, u64]
        lib.gen_instance_seed.restype = u64
        lib.gen_rng_stream.argtypes = [u64, ctypes.c_int64, ctypes.c_void_p]
        lib.gen_rng_below.argtypes = [u64, u64, ctypes.c_int64, ctypes.c_void_p]
        _lib = lib
    return _lib


def _arr(ptr, count, dtype):
    if count == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dtype, copy=True)


@dataclass
class Instance:
    """A CSP P=(X,D,C) in flat form.  Values of variable i are
    lo[i] .. lo[i]+dsize[i]-1; bit a of a domain word row stands for lo[i]+a."""
    lo: np.ndarray
    dsize: np.ndarray
    type: np.ndarray
    arity: np.ndarray
    var_off: np.ndarray
    vars: np.ndarray
    par_off: np.ndarray
    params: np.ndarray
    tab_off: np.ndarray
    tabs: np.ndarray
    init: np.ndarray | None = None   # optional n x W uint32 initial domain bits
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.lo.shape[0])

    @property
    def m(self) -> int:
        return int(self.type.shape[0])

    @property
    def dmax(self) -> int:
        return int(self.dsize.max()) if self.n else 1

    @property
    def W(self) -> int:
        return (self.dmax + 31) // 32

    def scope(self, c: int) -> np.ndarray:
        return self.vars[self.var_off[c]:self.var_off[c + 1]]

    def par(self, c: int) -> np.ndarray:
        return self.params[self.par_off[c]:self.par_off[c + 1]]

    def tab(self, c: int) -> np.ndarray:
        return self.tabs[self.tab_off[c]:self.tab_off[c + 1]]

    def with_init(self, init: np.ndarray | None) -> "Instance":
        """Copy with a restricted initial domain (n x W uint32 bit rows)."""
        out = Instance(**{k: getattr(self, k) for k in (
            "lo", "dsize", "type", "arity", "var_off", "vars", "par_off",
            "params", "tab_off", "tabs")}, init=None, name=self.name, meta=dict(self.meta))
        if init is not None:
            init = np.ascontiguousarray(init, dtype=np.uint32).reshape(self.n, self.W)
            out.init = init.copy()
        return out

    def with_gac(self) -> "Instance":
        """Copy whose all-different constraints are of the generalized-arc-
        consistency kind (same constraints, same solutions)."""
        out = self.with_init(self.init)
        out.type = np.where(self.type == ALLDIFF, ALLDIFF_GAC, self.type).astype(self.type.dtype)
        out.name = self.name + "_gac"
        return out

    def with_linear_ad(self) -> "Instance":
        """Copy whose linear <= constraints are propagated together with the
        all-different constraints inside their scopes (same constraints,
        same solutions)."""
        out = self.with_init(self.init)
        out.type = np.where(self.type == LINEAR_LE, LINEAR_LE_AD, self.type).astype(self.type.dtype)
        out.name = self.name + "_lad"
        return out

    def full_init(self) -> np.ndarray:
        """n x W bit rows of the full initial domains (all values allowed)."""
        W = self.W
        out = np.zeros((self.n, W), dtype=np.uint32)
        for i in range(self.n):
            d = int(self.dsize[i])
            for w in range(W):
                nb = min(32, max(0, d - 32 * w))
                out[i, w] = (1 << nb) - 1 if nb < 32 else 0xFFFFFFFF
        return out

    def fix(self, assignment: dict[int, int]) -> "Instance":
        """Copy whose initial domain of each var i in `assignment` is the single
        value assignment[i] (a sub-CSP of this instance)."""
        init = self.init.copy() if self.init is not None else self.full_init()
        for i, v in assignment.items():
            a = int(v) - int(self.lo[i])
            row = np.zeros(self.W, dtype=np.uint32)
            if 0 <= a < int(self.dsize[i]) and (int(init[i, a // 32]) >> (a % 32)) & 1:
                row[a // 32] = np.uint32(1 << (a % 32))
            init[i] = row
        return self.with_init(init)


def _wrap(p, name, meta) -> Instance:
    lib = _load()
    g = p.contents
    n, m = g.n, g.m
    var_off = _arr(g.var_off, m + 1, np.int64)
    par_off = _arr(g.par_off, m + 1, np.int64)
    tab_off = _arr(g.tab_off, m + 1, np.int64)
    inst = Instance(
        lo=_arr(g.lo, n, np.int32), dsize=_arr(g.dsize, n, np.int32),
        type=_arr(g.type, m, np.int32), arity=_arr(g.arity, m, np.int32),
        var_off=var_off, vars=_arr(g.vars, int(var_off[-1]), np.int32),
        par_off=par_off, params=_arr(g.params, int(par_off[-1]), np.int64),
        tab_off=tab_off, tabs=_arr(g.tabs, int(tab_off[-1]), np.uint32),
        name=name, meta=meta)
    lib.gen_free(p)
    return inst


def instance_seed(base: int, index: int) -> int:
    return int(_load().gen_instance_seed(base, index))


def rng_stream(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _load().gen_rng_stream(seed, count, out.ctypes.data)
    return out


def rng_below(seed: int, r: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _load().gen_rng_below(seed, r, count, out.ctypes.data)
    return out


def queens(n: int) -> Instance:
    return _wrap(_load().gen_queens(n), f"queens{n}", {"n": n})


def worked_example(form: int = 0) -> Instance:
    return _wrap(_load().gen_worked_example(form), f"worked_example_{form}", {"form": form})


def rb(index: int = 0, n: int = 40, d: int = 16, dens_pm: int = 250, tight_pm: int = 350,
       base: int = SEED_RB) -> Instance:
    seed = instance_seed(base, index)
    return _wrap(_load().gen_rb(seed, n, d, dens_pm, tight_pm), f"rb_n{n}_d{d}_i{index}",
                 {"seed": seed, "n": n, "d": d, "dens_pm": dens_pm, "tight_pm": tight_pm,
                  "index": index, "base": base})


SWEEP_RANGES = dict(nlo=20, nhi=120, dlo=8, dhi=64, plo=100, phi=300, tlo=200, thi=500)


def rb_sweep(index: int, base: int = SEED_SWEEP, **ranges) -> Instance:
    r = dict(SWEEP_RANGES)
    r.update(ranges)
    seed = instance_seed(base, index)
    p = _load().gen_rb_sweep(seed, r["nlo"], r["nhi"], r["dlo"], r["dhi"],
                             r["plo"], r["phi"], r["tlo"], r["thi"])
    return _wrap(p, f"sweep_{base}_{index}", {"seed": seed, "index": index, "base": base, **r})


def tree(index: int, n: int, d: int, tight_pm: int, base: int = 11) -> Instance:
    seed = instance_seed(base, index)
    return _wrap(_load().gen_tree(seed, n, d, tight_pm), f"tree_n{n}_d{d}_i{index}",
                 {"seed": seed, "n": n, "d": d, "tight_pm": tight_pm})


def global_family(index: int = 0, n: int = 200, lo: int = 0, d: int = 256, n_ad: int = 10,
                  k_ad: int = 20, n_lin: int = 30, lin_k: int = 0, amax: int = 9,
                  b_pm: int = 450, base: int = SEED_GLOBAL) -> Instance:
    seed = instance_seed(base, index)
    p = _load().gen_global(seed, n, lo, d, n_ad, k_ad, n_lin, lin_k, amax, b_pm)
    return _wrap(p, f"global_n{n}_d{d}_i{index}",
                 {"seed": seed, "n": n, "d": d, "n_ad": n_ad, "k_ad": k_ad, "n_lin": n_lin,
                  "lin_k": lin_k, "amax": amax, "b_pm": b_pm})


def global_twin(index: int = 0, n: int = 8, d: int = 8, k_ad: int = 5) -> Instance:
    """Scaled twin of the global family: n vars over 0..d-1, 2 all-different
    over k_ad vars, 3 linear <= over all vars with b = 45% of the maximum
    sum (small enough to enumerate exhaustively at the default size)."""
    return global_family(index, n=n, lo=0, d=d, n_ad=2, k_ad=k_ad, n_lin=3, lin_k=0,
                         amax=9, b_pm=450, base=SEED_GLOBAL + 100)


def mixed(index: int, n: int = 5, dmax: int = 5, m: int = 6, type_mask: int = 0x7F,
          base: int = 17) -> Instance:
    seed = instance_seed(base, index)
    return _wrap(_load().gen_mixed(seed, n, dmax, m, type_mask), f"mixed_{index}",
                 {"seed": seed, "n": n, "dmax": dmax, "m": m, "type_mask": type_mask})
