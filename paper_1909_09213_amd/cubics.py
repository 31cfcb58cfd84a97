"""Python binding of libcubics.so (ctypes).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory (solution buffers) and the stream.
Names follow the C ABI in include/cubics.h: ``cubics_create`` ->
:class:`Context`, ``cubics_load`` -> :meth:`Context.load`, ``cubics_solve`` ->
:meth:`Context.solve`, ``cubics_solve_batch`` -> :meth:`Context.solve_batch`,
``cubics_root`` -> :meth:`Context.root`.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcubics.so")

MODE_FIRST, MODE_ALL, MODE_COUNT = 0, 1, 2
LAYOUT_AUTO, LAYOUT_LANE, LAYOUT_SEG, LAYOUT_VAR = 0, 1, 2, 3
AUTOTUNE_DIVS = 3  # worker counts the autotuner tries: the maximum divided by 1, 2, 4
AUTOTUNE_DIV_VALUES = (1, 2, 4)
BRANCH_FIRST_FAIL, BRANCH_LEARNED = 0, 1
VERDICTS = {0: "SAT", 1: "UNSAT", 2: "LIMIT", 3: "CANCELLED"}
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED"}


class CubicsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Limits(ctypes.Structure):
    _fields_ = [
        ("max_nodes", ctypes.c_uint64), ("max_solutions", ctypes.c_uint64),
        ("time_ms", ctypes.c_int64), ("branching", ctypes.c_int32), ("layout", ctypes.c_int32),
        ("split_target", ctypes.c_int64), ("sol_buf", ctypes.c_void_p),
        ("sol_capacity", ctypes.c_uint64), ("workers", ctypes.c_int32), ("donate", ctypes.c_int32),
        ("policy", ctypes.c_void_p), ("tables_in_lds", ctypes.c_int32), ("explore_pm", ctypes.c_int32),
        ("trace_buf", ctypes.c_void_p), ("trace_capacity", ctypes.c_uint64), ("seed", ctypes.c_uint32),
        ("use_graph", ctypes.c_int32), ("two_way", ctypes.c_int32),
        ("active_per_xcd", ctypes.c_int32), ("value_policy", ctypes.c_void_p),
    ]


class LnsParams(ctypes.Structure):
    _fields_ = [("neighborhoods", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("relax_pm", ctypes.c_int32), ("seed", ctypes.c_uint32),
                ("max_nodes", ctypes.c_uint64), ("time_ms", ctypes.c_int64)]


class LnsResult(ctypes.Structure):
    _fields_ = [("objective", ctypes.c_int64), ("found", ctypes.c_int32), ("optimal", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("improvements", ctypes.c_int32),
                ("nodes", ctypes.c_uint64), ("ms", ctypes.c_double)]


class _Result(ctypes.Structure):
    _fields_ = [
        ("verdict", ctypes.c_int32), ("truncated", ctypes.c_int32),
        ("count", ctypes.c_uint64), ("n_written", ctypes.c_uint64), ("nodes", ctypes.c_uint64),
        ("fails", ctypes.c_uint64), ("revisions", ctypes.c_uint64), ("steals", ctypes.c_uint64),
        ("alg_bytes", ctypes.c_uint64), ("tasks", ctypes.c_uint64), ("traces", ctypes.c_uint64),
        ("ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
    ]


@dataclass
class Result:
    verdict: str
    count: int
    n_written: int
    nodes: int
    fails: int
    revisions: int
    steals: int
    alg_bytes: int
    tasks: int
    traces: int
    truncated: bool
    ms: float
    kernel_ms: float
    solutions: np.ndarray | None = None


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libcubics.so; raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libcubics.so not built at {path}; run __graft_entry__.build()")
    # Load torch first: its bundled HIP runtime (same soname libamdhip64.so.7)
    # then serves libcubics too, so the process holds a single HIP runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.cubics_last_error.restype = ctypes.c_char_p
    lib.cubics_create.argtypes = [i32, vp, ctypes.POINTER(vp)]
    lib.cubics_destroy.argtypes = [vp]
    lib.cubics_destroy.restype = None
    lib.cubics_set_stream.argtypes = [vp, vp]
    lib.cubics_cancel.argtypes = [vp]
    lib.cubics_cancel.restype = None
    lib.cubics_load.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.cubics_lns.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                               ctypes.POINTER(LnsParams), vp, ctypes.POINTER(LnsResult)]
    lib.cubics_lns.restype = ctypes.c_int
    lib.cubics_free.argtypes = [vp]
    lib.cubics_free.restype = None
    lib.cubics_prob_info.argtypes = [vp] + [ctypes.POINTER(i32)] * 4
    lib.cubics_root.argtypes = [vp, i32, vp, ctypes.POINTER(i32)]
    lib.cubics_features.argtypes = [vp, vp, i32, vp]
    lib.cubics_value_features.argtypes = [vp, vp, i32, i32, vp]
    lib.cubics_solve.argtypes = [vp, i32, ctypes.POINTER(Limits), ctypes.POINTER(_Result)]
    lib.cubics_solve_batch.argtypes = [vp, i32, i32, ctypes.POINTER(Limits), ctypes.POINTER(_Result)]
    lib.cubics_solve_batch_static.argtypes = [vp, i32, i32, ctypes.POINTER(Limits), ctypes.POINTER(_Result)]
    lib.cubics_autotune.argtypes = [vp, i32, i32, ctypes.POINTER(Limits), i64, ctypes.POINTER(i32),
                                    ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    lib.cubics_policy_create.argtypes = [vp, vp, ctypes.POINTER(vp)]
    lib.cubics_policy_free.argtypes = [vp]
    lib.cubics_policy_free.restype = None
    lib.cubics_policy_get.argtypes = [vp, vp]
    lib.cubics_policy_set.argtypes = [vp, vp]
    lib.cubics_mlp_forward.argtypes = [vp, vp, i32, i64, vp]
    lib.cubics_mlp_grad.argtypes = [vp, vp, i32, vp, i32, i64, vp, vp]
    lib.cubics_mlp_train_step.argtypes = [vp, vp, i32, vp, i32, i64, ctypes.c_float, i32, vp]
    for f in ("cubics_create", "cubics_set_stream", "cubics_load", "cubics_prob_info",
              "cubics_root", "cubics_features", "cubics_value_features", "cubics_solve", "cubics_solve_batch",
              "cubics_solve_batch_static", "cubics_autotune", "cubics_policy_create",
              "cubics_policy_get", "cubics_policy_set", "cubics_mlp_forward", "cubics_mlp_grad",
              "cubics_mlp_train_step"):
        getattr(lib, f).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        msg = _lib.cubics_last_error().decode()
        raise CubicsError(rc, msg)


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


class Problem:
    """A CSP loaded on the device (owns the device copy)."""

    def __init__(self, ctx, handle, inst):
        self.ctx = ctx
        self.handle = handle
        self.n = inst.n
        self.W_in = inst.W                  # words per row of the caller's bit rows
        self.W = self.info()["W"]           # words per domain on the device (>= W_in)
        self.lo = np.asarray(inst.lo, dtype=np.int32).copy()
        self.dsize = np.asarray(inst.dsize, dtype=np.int32).copy()
        self.name = getattr(inst, "name", "")

    def info(self):
        v = [ctypes.c_int32() for _ in range(4)]
        _check(_lib.cubics_prob_info(self.handle, *[ctypes.byref(x) for x in v]))
        return {"n": v[0].value, "W": v[1].value, "n_units": v[2].value, "n_global": v[3].value}

    def free(self):
        if self.handle:
            _lib.cubics_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _torch():
    import torch
    return torch


class Context:
    """cubics_create on `device`, using torch's current stream on that device."""

    def __init__(self, device: int = 0, stream=None):
        lib = load_library()
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("cubics needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = device
        self.torch_device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.cubics_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            _lib.cubics_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cancel(self):
        _lib.cubics_cancel(self.handle)

    # ---------------------------------------------------------------- load
    @staticmethod
    def _arrays(inst):
        return dict(
            lo=np.ascontiguousarray(inst.lo, dtype=np.int32),
            dsize=np.ascontiguousarray(inst.dsize, dtype=np.int32),
            type=np.ascontiguousarray(inst.type, dtype=np.int32),
            arity=np.ascontiguousarray(inst.arity, dtype=np.int32),
            var_off=np.ascontiguousarray(inst.var_off, dtype=np.int64),
            vars=np.ascontiguousarray(inst.vars, dtype=np.int32),
            par_off=np.ascontiguousarray(inst.par_off, dtype=np.int64),
            params=np.ascontiguousarray(inst.params, dtype=np.int64),
            tab_off=np.ascontiguousarray(inst.tab_off, dtype=np.int64),
            tabs=np.ascontiguousarray(inst.tabs, dtype=np.uint32),
        )

    def load(self, inst) -> Problem:
        keep = self._arrays(inst)
        init = None if inst.init is None else np.ascontiguousarray(inst.init, dtype=np.uint32)
        h = ctypes.c_void_p()
        _check(_lib.cubics_load(
            self.handle, inst.n, _ptr(keep["lo"]), _ptr(keep["dsize"]), _ptr(init), inst.m,
            _ptr(keep["type"]), _ptr(keep["arity"]), _ptr(keep["var_off"]), _ptr(keep["vars"]),
            _ptr(keep["par_off"]), _ptr(keep["params"]), _ptr(keep["tab_off"]), _ptr(keep["tabs"]),
            ctypes.byref(h)))
        return Problem(self, h, inst)

    def lns(self, inst, obj, *, neighborhoods: int = 256, rounds: int = 0, relax_pm: int = 300,
            max_nodes: int = 100_000, time_ms: int = 0, seed: int = 1) -> dict:
        """cubics_lns: minimise sum obj[i] * x_i over the solutions of inst."""
        keep = self._arrays(inst)
        init = None if inst.init is None else np.ascontiguousarray(inst.init, dtype=np.uint32)
        ob = np.ascontiguousarray(obj, dtype=np.int64)
        if ob.shape != (inst.n,):
            raise ValueError("obj must have one coefficient per variable")
        best = np.zeros(max(inst.n, 1), dtype=np.int32)
        lp = LnsParams(neighborhoods, rounds, relax_pm, seed, max_nodes, time_ms)
        r = LnsResult()
        _check(_lib.cubics_lns(
            self.handle, inst.n, _ptr(keep["lo"]), _ptr(keep["dsize"]), _ptr(init), inst.m,
            _ptr(keep["type"]), _ptr(keep["arity"]), _ptr(keep["var_off"]), _ptr(keep["vars"]),
            _ptr(keep["par_off"]), _ptr(keep["params"]), _ptr(keep["tab_off"]), _ptr(keep["tabs"]),
            _ptr(ob), ctypes.byref(lp), best.ctypes.data, ctypes.byref(r)))
        return {"best": best[:inst.n].copy() if r.found else None, "objective": int(r.objective),
                "found": bool(r.found), "optimal": bool(r.optimal), "rounds": int(r.rounds),
                "improvements": int(r.improvements), "nodes": int(r.nodes), "ms": float(r.ms)}

    # ------------------------------------------------------------ autotune
    def autotune(self, probs, mode: int = MODE_COUNT, time_ms: int = 50, rates: bool = False, **kw):
        """cubics_autotune: returns the chosen layout (1 LANE, 2 SEG, 3 VAR);
        with rates=True, (layout, worker divisor, {(layout, divisor): nodes
        per ms}) for every pair tried; self.last_active_per_xcd keeps the
        chosen instances per XCD queue (0 = one queue)."""
        B = len(probs)
        arr = (ctypes.c_void_p * B)(*[p.handle for p in probs])
        lims = (Limits * B)()
        for b in range(B):
            L = Limits()
            L.donate = 1 if kw.get("donate", True) else 0
            L.split_target = kw.get("split_target", 0)
            L.max_nodes = kw.get("max_nodes", 0)
            L.active_per_xcd = kw.get("active_per_xcd", 0)
            lims[b] = L
        chosen, div, act = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        rt = (ctypes.c_double * (3 * AUTOTUNE_DIVS))()
        _check(_lib.cubics_autotune(arr, B, mode, lims, time_ms, ctypes.byref(chosen), ctypes.byref(div),
                                    ctypes.byref(act), rt))
        self.last_active_per_xcd = act.value
        if rates:
            table = {(k // AUTOTUNE_DIVS + 1, AUTOTUNE_DIV_VALUES[k % AUTOTUNE_DIVS]): rt[k]
                     for k in range(3 * AUTOTUNE_DIVS) if rt[k] > 0}
            return chosen.value, div.value, table
        return chosen.value

    # ---------------------------------------------------------------- root
    def root(self, prob: Problem, layout: int = LAYOUT_AUTO, device_words: bool = False):
        """cubics_root: (failed, domains [n, W]); W = the caller's words per
        domain, or the device's (which may be wider) with device_words."""
        out = np.zeros((max(prob.n, 1), prob.W), dtype=np.uint32)
        failed = ctypes.c_int32()
        _check(_lib.cubics_root(prob.handle, layout, out.ctypes.data, ctypes.byref(failed)))
        return bool(failed.value), out[:prob.n, :(prob.W if device_words else prob.W_in)].copy()

    def features(self, prob: Problem, dom=None, depth: int = 0) -> np.ndarray:
        """cubics_features: [n, 5] policy features at a node with domains dom
        ([n, W] device words, as root(..., device_words=True) returns; None =
        the initial domains) and the given depth."""
        out = np.zeros((max(prob.n, 1), 5), dtype=np.float32)
        ptr = None
        if dom is not None:
            dom = np.ascontiguousarray(dom, dtype=np.uint32)
            if dom.shape != (prob.n, prob.W):
                raise ValueError(f"dom must have shape {(prob.n, prob.W)}")
            ptr = dom.ctypes.data
        _check(_lib.cubics_features(prob.handle, ptr, depth, out.ctypes.data))
        return out[:prob.n].copy()

    def value_features(self, prob: Problem, dom=None, depth: int = 0, x: int = 0) -> np.ndarray:
        """cubics_value_features: [32 W, 5] features of the values of x at a
        node with domains dom ([n, W] device words; None = the initial
        domains) and the given depth."""
        nv = 32 * prob.W
        out = np.zeros((nv, 5), dtype=np.float32)
        ptr = None
        if dom is not None:
            dom = np.ascontiguousarray(dom, dtype=np.uint32)
            if dom.shape != (prob.n, prob.W):
                raise ValueError(f"dom must have shape {(prob.n, prob.W)}")
            ptr = dom.ctypes.data
        _check(_lib.cubics_value_features(prob.handle, ptr, depth, x, out.ctypes.data))
        return out

    # --------------------------------------------------------------- solve
    def _limits(self, prob, mode, max_nodes, max_solutions, time_ms, branching, layout,
                split_target, sol_capacity, workers, donate, policy, tables_in_lds=0,
                trace=None, explore_pm=0, seed=0, use_graph=False, two_way=False,
                no_buffer=False, value_policy=None):
        torch = _torch()
        L = Limits()
        L.max_nodes = max_nodes
        L.max_solutions = max_solutions
        L.time_ms = time_ms
        L.branching = branching
        L.layout = layout
        L.split_target = split_target
        L.workers = workers
        L.donate = 1 if donate else 0
        L.policy = policy.handle if policy is not None else None
        L.value_policy = value_policy.handle if value_policy is not None else None
        L.tables_in_lds = tables_in_lds
        L.use_graph = 1 if use_graph else 0
        L.two_way = 1 if two_way else 0
        if trace is not None:
            L.trace_buf = trace.data_ptr()
            L.trace_capacity = trace.shape[0]
            L.explore_pm = explore_pm
            L.seed = seed
        buf = None
        if mode == MODE_FIRST and sol_capacity == 0 and not no_buffer:
            sol_capacity = 1
        if sol_capacity > 0 and prob.n > 0:
            buf = torch.empty((sol_capacity, prob.n), dtype=torch.int32, device=self.torch_device)
            L.sol_buf = buf.data_ptr()
            L.sol_capacity = sol_capacity
        return L, buf

    @staticmethod
    def _result(r: _Result, buf, n) -> Result:
        sols = None
        if buf is not None:
            sols = buf[: int(r.n_written)].cpu().numpy()
        elif n == 0 and r.count > 0:
            sols = np.zeros((int(min(r.n_written, 1)), 0), dtype=np.int32)
        return Result(VERDICTS.get(r.verdict, str(r.verdict)), int(r.count), int(r.n_written),
                      int(r.nodes), int(r.fails), int(r.revisions), int(r.steals), int(r.alg_bytes),
                      int(r.tasks), int(r.traces), bool(r.truncated), float(r.ms), float(r.kernel_ms), sols)

    def solve(self, prob: Problem, mode: int = MODE_COUNT, *, max_nodes: int = 0,
              max_solutions: int = 0, time_ms: int = 0, branching: int = BRANCH_FIRST_FAIL,
              layout: int = LAYOUT_AUTO, split_target: int = 0, sol_capacity: int = 0,
              workers: int = 0, donate: bool = True, policy=None, tables_in_lds: int = 0,
              use_graph: bool = False, two_way: bool = False, value_policy=None) -> Result:
        L, buf = self._limits(prob, mode, max_nodes, max_solutions, time_ms, branching, layout,
                              split_target, sol_capacity, workers, donate, policy, tables_in_lds,
                              use_graph=use_graph, two_way=two_way, value_policy=value_policy)
        r = _Result()
        _check(_lib.cubics_solve(prob.handle, mode, ctypes.byref(L), ctypes.byref(r)))
        return self._result(r, buf, prob.n)

    def solve_batch(self, probs, mode: int = MODE_FIRST, *, max_nodes: int = 0,
                    max_solutions: int = 0, time_ms: int = 0, branching: int = BRANCH_FIRST_FAIL,
                    layout: int = LAYOUT_AUTO, split_target: int = 0, sol_capacity: int = 0,
                    workers: int = 0, donate: bool = True, policy=None, trace=None,
                    explore_pm: int = 0, seed: int = 0, use_graph: bool = False,
                    two_way: bool = False, sol_out=None, static_scratch: bool = False,
                    active_per_xcd: int = 0, value_policy=None):
        """trace: optional torch float32 cuda tensor [cap, 8] receiving trace records.
        sol_out: optional int32 cuda tensor [B, >= max n]; FIRST mode stores
        instance b's solution in row b (no per-instance buffers, and the
        results carry no solutions: read them from sol_out).
        static_scratch: call cubics_solve_batch_static (the allocation-free
        variant) instead of cubics_solve_batch."""
        B = len(probs)
        arr = (ctypes.c_void_p * B)(*[p.handle for p in probs])
        lims = (Limits * B)()
        bufs = []
        if sol_out is not None:
            if mode != MODE_FIRST or sol_out.dtype != _torch().int32 or sol_out.dim() != 2 \
                    or sol_out.shape[0] < B or sol_out.shape[1] < max(p.n for p in probs) \
                    or not sol_out.is_cuda or not sol_out.is_contiguous():
                raise ValueError("sol_out: FIRST mode and a contiguous int32 cuda tensor [B, max n]")
            row = sol_out.shape[1] * 4
            base = sol_out.data_ptr()
        for b, p in enumerate(probs):
            L, buf = self._limits(p, mode, max_nodes, max_solutions, time_ms, branching, layout,
                                  split_target, 0 if sol_out is not None else sol_capacity,
                                  workers, donate, policy, 0,
                                  trace if b == 0 else None, explore_pm, seed, use_graph, two_way,
                                  no_buffer=sol_out is not None, value_policy=value_policy)
            if sol_out is not None:
                L.sol_buf = base + b * row
                L.sol_capacity = 1
            L.active_per_xcd = active_per_xcd
            lims[b] = L
            bufs.append(buf)
        res = (_Result * B)()
        fn = _lib.cubics_solve_batch_static if static_scratch else _lib.cubics_solve_batch
        _check(fn(arr, B, mode, lims, res))
        return [self._result(res[b], bufs[b], probs[b].n) for b in range(B)]


class Policy:
    """cubics_policy: the branching network's parameters on the device.

    theta: 449 float32 values = W1[64][5], b1[64], w2[64], b2 (fp32 master)."""

    NP = 449

    def __init__(self, ctx: Context, theta):
        self.ctx = ctx
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.shape == (self.NP,)
        h = ctypes.c_void_p()
        _check(_lib.cubics_policy_create(ctx.handle, th.ctypes.data, ctypes.byref(h)))
        self.handle = h

    def get(self) -> np.ndarray:
        out = np.zeros(self.NP, dtype=np.float32)
        _check(_lib.cubics_policy_get(self.handle, out.ctypes.data))
        return out

    def set(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        _check(_lib.cubics_policy_set(self.handle, th.ctypes.data))

    def forward(self, rec):
        """rec: float32 cuda tensor [N, ld >= 5] (features in columns 0..4)."""
        torch = _torch()
        assert rec.dtype == torch.float32 and rec.is_contiguous()
        N, ld = rec.shape
        y = torch.empty(N, dtype=torch.float32, device=rec.device)
        _check(_lib.cubics_mlp_forward(self.handle, rec.data_ptr(), ld, N, y.data_ptr()))
        return y

    def grad(self, rec, target_col: int = 7):
        """Gradient of the MSE with targets rec[:, target_col] (trace records)."""
        torch = _torch()
        N, ld = rec.shape
        g = torch.empty(self.NP, dtype=torch.float32, device=rec.device)
        loss = torch.empty(1, dtype=torch.float32, device=rec.device)
        _check(_lib.cubics_mlp_grad(self.handle, rec.data_ptr(), ld,
                                    rec.data_ptr() + 4 * target_col, ld, N,
                                    g.data_ptr(), loss.data_ptr()))
        return g, loss

    def train_step(self, rec, lr: float, step: int, target_col: int = 7) -> float:
        N, ld = rec.shape
        loss = ctypes.c_float()
        _check(_lib.cubics_mlp_train_step(self.handle, rec.data_ptr(), ld,
                                          rec.data_ptr() + 4 * target_col, ld, N, lr, step,
                                          ctypes.byref(loss)))
        return float(loss.value)

    def close(self):
        if self.handle:
            _lib.cubics_policy_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
