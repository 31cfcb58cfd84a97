"""CPU oracle - TEST INFRASTRUCTURE ONLY.

Python access to the plain single-threaded reference solver in ``oracle.c``
(AC-3 style propagation plus chronological d-way backtracking with first-fail)
and to ``mlp_ref.py`` (fp64 reference of the branching network).  Only the
tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg import
this package; the GPU library never does, and the two share no code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

MODE_FIRST, MODE_ALL, MODE_COUNT = 0, 1, 2
VERDICTS = {0: "SAT", 1: "UNSAT", 2: "LIMIT"}


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc -O2)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp,
                               os.path.join(_HERE, "oracle.c")])
        os.replace(tmp, _SO)
    return _SO


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("m", ctypes.c_int32),
        ("lo", ctypes.c_void_p), ("dsize", ctypes.c_void_p), ("init", ctypes.c_void_p),
        ("type", ctypes.c_void_p), ("arity", ctypes.c_void_p),
        ("var_off", ctypes.c_void_p), ("vars", ctypes.c_void_p),
        ("par_off", ctypes.c_void_p), ("params", ctypes.c_void_p),
        ("tab_off", ctypes.c_void_p), ("tabs", ctypes.c_void_p),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [("verdict", ctypes.c_int32), ("truncated", ctypes.c_int32),
                ("count", ctypes.c_int64), ("n_written", ctypes.c_int64),
                ("nodes", ctypes.c_int64), ("fails", ctypes.c_int64),
                ("revisions", ctypes.c_int64), ("max_depth", ctypes.c_int64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        PP = ctypes.POINTER(_Problem)
        lib.orc_solve.argtypes = [PP, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(_Stats)]
        lib.orc_solve.restype = ctypes.c_int
        lib.orc_solve2.argtypes = [PP, ctypes.c_int, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_Stats)]
        lib.orc_solve2.restype = ctypes.c_int
        lib.orc_root.argtypes = [PP, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_root.restype = ctypes.c_int
        lib.orc_verify.argtypes = [PP, ctypes.c_void_p]
        lib.orc_verify.restype = ctypes.c_int
        lib.orc_brute.argtypes = [PP, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64]
        lib.orc_brute.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _problem(inst):
    """Build the C view of a cspgen.Instance; returns (struct, keepalive)."""
    keep = {
        "lo": np.ascontiguousarray(inst.lo, dtype=np.int32),
        "dsize": np.ascontiguousarray(inst.dsize, dtype=np.int32),
        "type": np.ascontiguousarray(inst.type, dtype=np.int32),
        "arity": np.ascontiguousarray(inst.arity, dtype=np.int32),
        "var_off": np.ascontiguousarray(inst.var_off, dtype=np.int64),
        "vars": np.ascontiguousarray(inst.vars, dtype=np.int32),
        "par_off": np.ascontiguousarray(inst.par_off, dtype=np.int64),
        "params": np.ascontiguousarray(inst.params, dtype=np.int64),
        "tab_off": np.ascontiguousarray(inst.tab_off, dtype=np.int64),
        "tabs": np.ascontiguousarray(inst.tabs, dtype=np.uint32),
    }
    if inst.init is not None:
        keep["init"] = np.ascontiguousarray(inst.init, dtype=np.uint32)
    P = _Problem()
    P.n, P.m = inst.n, inst.m
    for k, a in keep.items():
        setattr(P, k, a.ctypes.data if a.size else None)
    if inst.init is None:
        P.init = None
    return P, keep


@dataclass
class Result:
    verdict: str
    count: int
    n_written: int
    nodes: int
    fails: int
    revisions: int
    max_depth: int
    truncated: bool
    solutions: np.ndarray  # n_written x n int32 values


def solve(inst, mode: int = MODE_COUNT, max_nodes: int = 0, cap: int = 0,
          sol_cap: int = 0, two_way: bool = False) -> Result:
    """two_way: 2-way branching (x = min D_x, then x != min D_x)."""
    lib = _load()
    P, keep = _problem(inst)
    sols = np.zeros((max(sol_cap, 0), max(inst.n, 1)), dtype=np.int32)
    st = _Stats()
    r = lib.orc_solve2(ctypes.byref(P), mode, max_nodes, cap,
                       sols.ctypes.data if sol_cap > 0 else None, sol_cap, 1 if two_way else 0,
                       ctypes.byref(st))
    if r != 0:
        raise ValueError("oracle: malformed instance")
    return Result(VERDICTS[st.verdict], st.count, st.n_written, st.nodes, st.fails,
                  st.revisions, st.max_depth, bool(st.truncated),
                  sols[:st.n_written, :inst.n].copy())


def root(inst):
    """Root fixpoint: (failed, n x W uint32 bit rows, revisions)."""
    lib = _load()
    P, keep = _problem(inst)
    out = np.zeros((max(inst.n, 1), inst.W), dtype=np.uint32)
    rev = ctypes.c_int64(0)
    r = lib.orc_root(ctypes.byref(P), out.ctypes.data, ctypes.byref(rev))
    if r < 0:
        raise ValueError("oracle: malformed instance")
    return bool(r), out[:inst.n].copy(), rev.value


def verify(inst, assignment) -> bool:
    lib = _load()
    P, keep = _problem(inst)
    x = np.ascontiguousarray(assignment, dtype=np.int32)
    assert x.shape[0] == inst.n
    return bool(lib.orc_verify(ctypes.byref(P), x.ctypes.data if x.size else None))


def brute(inst, limit: int = 10 ** 7, sol_cap: int = 0):
    """(count, solutions) by exhaustive enumeration; None if too large."""
    lib = _load()
    P, keep = _problem(inst)
    sols = np.zeros((max(sol_cap, 1), max(inst.n, 1)), dtype=np.int32)
    c = lib.orc_brute(ctypes.byref(P), limit, sols.ctypes.data if sol_cap > 0 else None, sol_cap)
    if c < 0:
        return None
    return int(c), sols[:min(c, sol_cap), :inst.n].copy()
