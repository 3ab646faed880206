"""Thin Python binding of libpa.so (ctypes).  Argument marshalling only: every
step of plotting and multiplication runs in the library's HIP kernels.  Device
memory and streams come from PyTorch (ROCm).  The binding fails loudly when
the library is missing; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpa.so")

PA_OK, PA_EINVAL, PA_ENOMEM, PA_EHIP, PA_EUNSUPPORTED = 0, 1, 2, 3, 4
ORDER_GREEDY, ORDER_EXHAUSTIVE, ORDER_LEARNED, ORDER_GIVEN = 0, 1, 2, 3
OPKIND_BITS, OPKIND_STREAM_K, OPKIND_STREAM_W, OPKIND_GEMM, OPKIND_FILL = 0, 1, 2, 10, 20
OPKIND_GATHER, OPKIND_COUNT, OPKIND_ROWLIST, OPKIND_FUSED, OPKIND_PLOT, OPKIND_PERSIST = 25, 26, 27, 28, 30, 40
PLOT_FP32_ESCALATE, PLOT_FP64 = 0, 1
RULE_CORNER, RULE_CENTER = 0, 1
TARGET_EQ, TARGET_LE, TARGET_LT = 0, 1, 2
MAX_DIMS, MAX_RELATIONS = 12, 32
MODEL_FEATURES = 16

STATUS_NAMES = {0: "PA_OK", 1: "PA_EINVAL", 2: "PA_ENOMEM", 3: "PA_EHIP", 4: "PA_EUNSUPPORTED"}


class PaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Axis(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_double), ("hi", ctypes.c_double), ("res", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Relation(ctypes.Structure):
    _fields_ = [("arity", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("vars", ctypes.POINTER(ctypes.c_int32)), ("coef", ctypes.POINTER(ctypes.c_double)),
                ("target", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BitArray(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("ndim", ctypes.c_int32), ("dims", ctypes.c_int32 * MAX_DIMS),
                ("row_words", ctypes.c_int64)]


class System(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("axes", ctypes.POINTER(Axis)),
                ("n_rel", ctypes.c_int32), ("rel", ctypes.POINTER(Relation))]


class Opts(ctypes.Structure):
    _fields_ = [("order_policy", ctypes.c_int32), ("n_given", ctypes.c_int32),
                ("given", ctypes.POINTER(ctypes.c_int32)), ("precision", ctypes.c_int32),
                ("audit", ctypes.c_int32), ("timing", ctypes.c_int32), ("plain", ctypes.c_int32),
                ("per_op", ctypes.c_int32), ("graph", ctypes.c_int32), ("single_launch", ctypes.c_int32),
                ("persist_wg", ctypes.c_int32),
                ("plot_strip", ctypes.c_int32), ("contract_units", ctypes.c_int32),
                ("model", ctypes.c_void_p), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("autotune", ctypes.c_int32), ("gemm_split", ctypes.c_int32), ("gemm_path", ctypes.c_int32),
                ("verify_order", ctypes.c_int32), ("sparse_pass", ctypes.c_int32),
                ("sparse_max_density", ctypes.c_int32), ("plot_rule", ctypes.c_int32),
                ("measure_density", ctypes.c_int32), ("tolerance", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("single_launch", ctypes.c_int32), ("persist_wg", ctypes.c_int32), ("plot_strip", ctypes.c_int32),
                ("contract_units", ctypes.c_int32), ("gemm_split", ctypes.c_int32), ("gemm_path", ctypes.c_int32),
                ("sparse_pass", ctypes.c_int32), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Report(ctypes.Structure):
    _fields_ = [("corners", ctypes.c_int64), ("corners_flagged", ctypes.c_int64),
                ("corners_disagree", ctypes.c_int64), ("corners_disagree_unflagged", ctypes.c_int64),
                ("nnz_out", ctypes.c_int64), ("n_steps", ctypes.c_int32), ("n_launches", ctypes.c_int32),
                ("merges", ctypes.c_int32 * (2 * MAX_RELATIONS)), ("cost_macs", ctypes.c_double),
                ("t_plot_ms", ctypes.c_double), ("t_contract_ms", ctypes.c_double), ("t_plan_ms", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "merges"}
        return d


_lib = None


def load(path: str = LIB_PATH):
    """Load libpa.so (built in-tree by paper_1609_00061_amd/build.py).  On a
    machine with a GPU, PyTorch's device runtime is initialised first: device
    memory and streams come from PyTorch, and its runtime does not start once
    the library has initialised HIP in the process."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libpa.so not built ({path}); run __graft_entry__.build() first")
    try:
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
    except ImportError:
        pass
    L = ctypes.CDLL(path)
    vp, i32p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)
    L.pa_row_words.argtypes = [ctypes.c_int32]
    L.pa_row_words.restype = ctypes.c_int64
    L.pa_array_words.argtypes = [ctypes.c_int32, i32p]
    L.pa_array_words.restype = ctypes.c_int64
    L.pa_last_error.restype = ctypes.c_char_p
    L.pa_plot_relation.argtypes = [ctypes.POINTER(Relation), ctypes.POINTER(Axis), ctypes.POINTER(Opts),
                                   ctypes.POINTER(BitArray), ctypes.POINTER(Report), vp]
    L.pa_contract.argtypes = [ctypes.POINTER(BitArray), i32p, ctypes.POINTER(BitArray), i32p, i32p, ctypes.c_int32,
                              ctypes.POINTER(BitArray), ctypes.POINTER(Opts), vp]
    L.pa_contract_noalloc.argtypes = L.pa_contract.argtypes
    L.pa_contract_count.argtypes = [ctypes.POINTER(BitArray), i32p, ctypes.POINTER(BitArray), i32p, i32p,
                                    ctypes.c_int32, vp, ctypes.POINTER(Opts), vp]
    L.pa_plan_create.argtypes = [ctypes.POINTER(System), i32p, ctypes.c_int32, ctypes.POINTER(Opts),
                                 ctypes.POINTER(vp)]
    L.pa_plan_execute.argtypes = [vp, ctypes.POINTER(BitArray), ctypes.POINTER(Report), vp]
    L.pa_plan_workspace_bytes.argtypes = [vp]
    L.pa_plan_workspace_bytes.restype = ctypes.c_size_t
    L.pa_plan_describe.argtypes = [ctypes.POINTER(System), i32p, ctypes.c_int32, ctypes.POINTER(Opts),
                                   ctypes.c_char_p, ctypes.c_int64]
    L.pa_plan_describe.restype = ctypes.c_int64
    L.pa_plan_destroy.argtypes = [vp]
    L.pa_plan_destroy.restype = None
    L.pa_solve_system.argtypes = [ctypes.POINTER(System), i32p, ctypes.c_int32, ctypes.POINTER(Opts),
                                  ctypes.POINTER(BitArray), ctypes.POINTER(Report), vp]
    L.pa_popcount.argtypes = [ctypes.POINTER(BitArray), ctypes.POINTER(ctypes.c_int64), vp]
    L.pa_tile_popcount.argtypes = [ctypes.POINTER(BitArray), ctypes.c_int32, ctypes.c_int32, vp, vp]
    L.pa_lds_read_rate.argtypes = [ctypes.POINTER(ctypes.c_double), vp]
    L.pa_plan_op_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
    L.pa_plan_op_times.restype = ctypes.c_int32
    L.pa_batch_create.argtypes = [ctypes.POINTER(System), ctypes.c_int32, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                  i32p, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    L.pa_batch_execute.argtypes = [vp, ctypes.POINTER(BitArray), ctypes.POINTER(Report), ctypes.POINTER(Report), vp]
    L.pa_batch_workspace_bytes.argtypes = [vp]
    L.pa_batch_workspace_bytes.restype = ctypes.c_size_t
    L.pa_batch_op_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int32]
    L.pa_batch_op_times.restype = ctypes.c_int32
    L.pa_batch_destroy.argtypes = [vp]
    L.pa_batch_destroy.restype = None
    L.pa_solve_batch.argtypes = [ctypes.POINTER(System), ctypes.c_int32, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                 i32p, ctypes.POINTER(Opts), ctypes.POINTER(BitArray), ctypes.POINTER(Report), vp]
    L.pa_workspace_bytes.argtypes = [ctypes.POINTER(System), i32p, ctypes.c_int32, ctypes.POINTER(Opts)]
    L.pa_workspace_bytes.restype = ctypes.c_size_t
    fp = ctypes.POINTER(ctypes.c_float)
    L.pa_model_n_params.restype = ctypes.c_int32
    L.pa_model_n_features.restype = ctypes.c_int32
    L.pa_model_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(vp)]
    L.pa_model_destroy.argtypes = [vp]
    L.pa_model_destroy.restype = None
    L.pa_model_get_params.argtypes = [vp, fp, ctypes.c_int32]
    L.pa_model_set_params.argtypes = [vp, fp, ctypes.c_int32]
    L.pa_model_forward.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    L.pa_model_set_level_cost.argtypes = [vp, ctypes.c_double]
    L.pa_model_gradient.argtypes = [vp, vp, vp, ctypes.c_int64, vp, fp, vp]
    L.pa_model_train_step.argtypes = [vp, vp, vp, ctypes.c_int64, ctypes.c_float, fp, vp]
    L.pa_model_save.argtypes = [vp, ctypes.c_char_p]
    L.pa_model_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(vp)]
    L.pa_step_features.argtypes = [ctypes.POINTER(System), i32p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32, fp]
    L.pa_plan_step_samples.argtypes = [vp, fp, fp, ctypes.c_int32]
    L.pa_plan_step_samples.restype = ctypes.c_int32
    for fn in (L.pa_plan_time_groups, L.pa_batch_time_groups):
        fn.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                       ctypes.POINTER(ctypes.c_double), ctypes.c_int32, vp]
        fn.restype = ctypes.c_int32
    for fn in (L.pa_plan_set_wait_limit, L.pa_batch_set_wait_limit):
        fn.argtypes = [vp, ctypes.c_int64]
    L.pa_autotune.argtypes = [ctypes.POINTER(System), ctypes.c_int32, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                              i32p, ctypes.POINTER(Opts), ctypes.c_int32, ctypes.POINTER(Tuning),
                              ctypes.POINTER(Tuning), ctypes.c_int32, i32p, vp]
    _lib = L
    return L


def _check(rc):
    if rc != PA_OK:
        raise PaError(rc, load().pa_last_error().decode())


def row_words(d: int) -> int:
    return int(load().pa_row_words(d))


def array_words(dims: Sequence[int]) -> int:
    arr = (ctypes.c_int32 * max(1, len(dims)))(*dims)
    return int(load().pa_array_words(len(dims), arr))


# ------------------------------------------------------------ marshalling
class _Keep:
    """Holds ctypes buffers alive for the duration of a call."""

    def __init__(self):
        self.items = []

    def i32(self, seq):
        a = (ctypes.c_int32 * max(1, len(seq)))(*[int(x) for x in seq])
        self.items.append(a)
        return a

    def f64(self, seq):
        arr = np.ascontiguousarray(np.asarray(seq, dtype=np.float64))
        self.items.append(arr)
        return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _relation(keep, rel, var_map=None) -> Relation:
    vs = list(rel.vars) if var_map is None else [var_map[v] for v in rel.vars]
    return Relation(len(vs), int(rel.degree), keep.i32(vs), keep.f64(rel.coef), int(getattr(rel, "target", 0)), 0)


def _system(keep, system) -> System:
    axes = (Axis * len(system.axes))(*[Axis(float(lo), float(hi), int(r), 0) for lo, hi, r in system.axes])
    rels = (Relation * len(system.relations))(*[_relation(keep, r) for r in system.relations])
    keep.items += [axes, rels]
    return System(len(system.axes), axes, len(system.relations), rels)


def make_opts(order=ORDER_EXHAUSTIVE, precision=PLOT_FP32_ESCALATE, audit=False, timing=False, plain=False,
              given: Optional[Sequence[int]] = None, model=None, keep: Optional[_Keep] = None, per_op=False,
              graph=False, single_launch=False, persist_wg=0, plot_strip=0, contract_units=0,
              autotune=False, gemm_split=0, gemm_path=0, verify_order=False, sparse_pass=0,
              sparse_max_density=0, workspace=None, plot_rule=RULE_CORNER, tolerance=0.0,
              measure_density=False) -> Opts:
    """pa_opts from keyword arguments; `workspace` is a device tensor the
    caller owns (its data pointer and byte size are passed)."""
    o = Opts()
    o.order_policy = order
    o.precision = precision
    o.audit = int(audit)
    o.timing = int(timing)
    o.plain = int(plain)
    o.per_op = int(per_op)
    o.graph = int(graph)
    o.single_launch = int(single_launch)
    o.persist_wg = int(persist_wg)
    o.plot_strip = int(plot_strip)
    o.contract_units = int(contract_units)
    o.autotune = int(autotune)
    o.gemm_split = int(gemm_split)
    o.gemm_path = int(gemm_path)
    o.verify_order = int(verify_order)
    o.sparse_pass = int(sparse_pass)
    o.sparse_max_density = int(sparse_max_density)
    o.plot_rule = int(plot_rule)
    o.tolerance = float(tolerance)
    o.measure_density = int(measure_density)
    if workspace is not None:
        o.workspace = ctypes.c_void_p(workspace.data_ptr())
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    if given is not None:
        assert keep is not None
        o.n_given = len(given) // 2
        o.given = keep.i32(given)
    if model is not None:
        h = model.handle if hasattr(model, "handle") else model
        o.model = h.value if isinstance(h, ctypes.c_void_p) else h
    return o


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def empty_bits(dims: Sequence[int], device="cuda"):
    """Device buffer (torch int32) for a bit array with the given dims."""
    import torch
    return torch.zeros(array_words(dims), dtype=torch.int32, device=device)


def bitarray(t, dims: Sequence[int]) -> BitArray:
    b = BitArray()
    b.data = ctypes.c_void_p(t.data_ptr())
    b.ndim = len(dims)
    for i, d in enumerate(dims):
        b.dims[i] = int(d)
    b.row_words = row_words(dims[-1]) if len(dims) else 1
    return b


# ---------------------------------------------------------- host helpers
def unpack_bits(words: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """Host-side view: packed words -> one byte per entry (for reading results)."""
    w = np.ascontiguousarray(np.asarray(words).view(np.uint32))
    if len(dims) == 0:
        return np.array(w[0] & 1, dtype=np.uint8)
    rw = row_words(dims[-1])
    rows = int(np.prod(dims[:-1])) if len(dims) > 1 else 1
    bits = np.unpackbits(w.reshape(rows, rw).view(np.uint8), axis=1, bitorder="little")
    return bits[:, :dims[-1]].reshape(tuple(dims)).astype(np.uint8)


def pack_bits(arr: np.ndarray) -> np.ndarray:
    """Host-side: one byte per entry -> packed int32 words (for passing inputs)."""
    arr = np.asarray(arr, dtype=np.uint8)
    dims = arr.shape
    if len(dims) == 0:
        return np.array([int(arr) & 1], dtype=np.uint32).view(np.int32)
    rw = row_words(dims[-1])
    rows = int(np.prod(dims[:-1])) if len(dims) > 1 else 1
    padded = np.zeros((rows, rw * 32), dtype=np.uint8)
    padded[:, :dims[-1]] = arr.reshape(rows, dims[-1])
    return np.packbits(padded, axis=1, bitorder="little").view(np.uint32).reshape(-1).view(np.int32)


# ------------------------------------------------------------ entry points
def plot_relation(rel, axes_of_vars, precision=PLOT_FP32_ESCALATE, audit=False, stream=None, report=True,
                  **exec_opts):
    """Plot one relation; returns (device words, dims, report dict or None)."""
    L = load()
    keep = _Keep()
    r = _relation(keep, rel, {v: i for i, v in enumerate(rel.vars)})
    axes = (Axis * len(axes_of_vars))(*[Axis(float(lo), float(hi), int(res), 0) for lo, hi, res in axes_of_vars])
    dims = [int(a[2]) for a in axes_of_vars]
    out = empty_bits(dims)
    ba = bitarray(out, dims)
    opts = make_opts(precision=precision, audit=audit, **exec_opts)
    rep = Report()
    _check(L.pa_plot_relation(ctypes.byref(r), axes, ctypes.byref(opts), ctypes.byref(ba),
                              ctypes.byref(rep) if report else None, _stream_ptr(stream)))
    return out, dims, (rep.as_dict() if report else None)


def contract(A, a_dims, a_vars, B, b_dims, b_vars, out_vars, out_dims, stream=None, plain=False, noalloc=False,
             out=None, **exec_opts):
    """C(out_vars) = OR over the other variables of A AND B (B may be None).
    noalloc: call pa_contract_noalloc (no device allocation by the library);
    out: the caller's output buffer (else a new one)."""
    L = load()
    keep = _Keep()
    C = empty_bits(out_dims) if out is None else out
    ba, bc = bitarray(A, a_dims), bitarray(C, out_dims)
    bb = bitarray(B, b_dims) if B is not None else None
    opts = make_opts(plain=plain, **exec_opts)
    fn = L.pa_contract_noalloc if noalloc else L.pa_contract
    _check(fn(ctypes.byref(ba), keep.i32(a_vars), ctypes.byref(bb) if bb is not None else None,
              keep.i32(b_vars if B is not None else []), keep.i32(out_vars), len(out_vars),
              ctypes.byref(bc), ctypes.byref(opts), _stream_ptr(stream)))
    return C


def contract_count(A, a_dims, a_vars, B, b_dims, b_vars, out_vars, out_dims, stream=None):
    """Counts (count semiring): C(out_vars) = number of entries of the other
    variables where A and B are both set (B may be None).  Returns a device
    int32 tensor holding the uint32 counts, row-major over out_dims."""
    import torch
    L = load()
    keep = _Keep()
    n = 1
    for d in out_dims:
        n *= int(d)
    C = torch.zeros(max(1, n), dtype=torch.int32, device="cuda")
    ba = bitarray(A, a_dims)
    bb = bitarray(B, b_dims) if B is not None else None
    opts = make_opts()
    _check(L.pa_contract_count(ctypes.byref(ba), keep.i32(a_vars), ctypes.byref(bb) if bb is not None else None,
                               keep.i32(b_vars if B is not None else []), keep.i32(out_vars), len(out_vars),
                               ctypes.c_void_p(C.data_ptr()), ctypes.byref(opts), _stream_ptr(stream)))
    return C


def describe_plan(system, exposed=None, order=ORDER_EXHAUSTIVE, precision=PLOT_FP32_ESCALATE,
                  given=None, plain=False, **exec_opts) -> dict:
    """Host-only: the plan (tree, layouts, kernels) as a dict."""
    L = load()
    keep = _Keep()
    exposed = list(system.exposed if exposed is None else exposed)
    s = _system(keep, system)
    opts = make_opts(order=order, precision=precision, given=given, plain=plain, keep=keep, **exec_opts)
    n = L.pa_plan_describe(ctypes.byref(s), keep.i32(exposed), len(exposed), ctypes.byref(opts), None, 0)
    buf = ctypes.create_string_buffer(int(n) + 1)
    L.pa_plan_describe(ctypes.byref(s), keep.i32(exposed), len(exposed), ctypes.byref(opts), buf, n + 1)
    return json.loads(buf.value.decode())


def _time_groups(fn, handle, reps, stream):
    cap = 4096
    ms = (ctypes.c_double * cap)()
    kd = (ctypes.c_int32 * cap)()
    mc = (ctypes.c_double * cap)()
    n = fn(handle, reps, ms, kd, mc, cap, _stream_ptr(stream))
    if n < 0:
        _check(PA_EINVAL)
    return [(int(kd[i]), float(ms[i]), float(mc[i])) for i in range(min(n, cap))]


class Plan:
    """A planned solve: pa_plan_create once, execute many times."""

    def __init__(self, system, exposed=None, order=ORDER_EXHAUSTIVE, precision=PLOT_FP32_ESCALATE, audit=False,
                 timing=False, plain=False, given=None, model=None, **exec_opts):
        L = load()
        self._keep = _Keep()
        self.exposed = list(system.exposed if exposed is None else exposed)
        self.dims = [int(system.axes[v][2]) for v in self.exposed]
        s = _system(self._keep, system)
        opts = make_opts(order=order, precision=precision, audit=audit, timing=timing, plain=plain, given=given,
                         model=model, keep=self._keep, **exec_opts)
        h = ctypes.c_void_p()
        _check(L.pa_plan_create(ctypes.byref(s), self._keep.i32(self.exposed), len(self.exposed),
                                ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h

    def workspace_bytes(self) -> int:
        return int(load().pa_plan_workspace_bytes(self.handle))

    def execute(self, out=None, stream=None, report=False):
        L = load()
        if out is None:
            out = empty_bits(self.dims)
        ba = bitarray(out, self.dims)
        rep = Report() if report else None
        _check(L.pa_plan_execute(self.handle, ctypes.byref(ba), ctypes.byref(rep) if report else None,
                                 _stream_ptr(stream)))
        return out, (rep.as_dict() if report else None), (list(rep.merges[:2 * 31]) if report else None)

    def op_times(self):
        """[(kind, ms, macs)] of the last execute (plan created with timing=2)."""
        L = load()
        cap = 256
        ms = (ctypes.c_double * cap)()
        kd = (ctypes.c_int32 * cap)()
        mc = (ctypes.c_double * cap)()
        n = L.pa_plan_op_times(self.handle, ms, kd, mc, cap)
        if n < 0:
            _check(PA_EINVAL)
        return [(int(kd[i]), float(ms[i]), float(mc[i])) for i in range(min(n, cap))]

    def time_groups(self, reps=20, stream=None):
        """[(kind, ms per launch, macs)] of every grouped launch, each timed
        over `reps` back-to-back launches (plan executed at least once)."""
        return _time_groups(load().pa_plan_time_groups, self.handle, reps, stream)

    def set_wait_limit(self, polls):
        """Bound of the single persistent launch's dependency waits (negative:
        give up at once; for tests of the failure path)."""
        _check(load().pa_plan_set_wait_limit(self.handle, int(polls)))

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.pa_plan_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


class Batch:
    """Many independent systems planned separately and executed together."""

    def __init__(self, systems, order=ORDER_EXHAUSTIVE, precision=PLOT_FP32_ESCALATE, audit=False, timing=False,
                 model=None, **exec_opts):
        L = load()
        self._keep = _Keep()
        self.systems = list(systems)
        self.dims = [[int(s.axes[v][2]) for v in s.exposed] for s in self.systems]
        arr = (System * len(self.systems))(*[_system(self._keep, s) for s in self.systems])
        exps = [self._keep.i32(list(s.exposed)) for s in self.systems]
        exp_ptrs = (ctypes.POINTER(ctypes.c_int32) * len(exps))(
            *[ctypes.cast(e, ctypes.POINTER(ctypes.c_int32)) for e in exps])
        n_exp = self._keep.i32([len(s.exposed) for s in self.systems])
        self._keep.items += [arr, exp_ptrs]
        opts = make_opts(order=order, precision=precision, audit=audit, timing=timing, model=model,
                         keep=self._keep, **exec_opts)
        h = ctypes.c_void_p()
        _check(L.pa_batch_create(arr, len(self.systems), exp_ptrs, n_exp, ctypes.byref(opts), ctypes.byref(h)))
        self.handle = h

    def workspace_bytes(self) -> int:
        return int(load().pa_batch_workspace_bytes(self.handle))

    def alloc_outputs(self):
        return [empty_bits(d) for d in self.dims]

    def execute(self, outs=None, stream=None, report=False, per_system=False):
        """Returns (outs, report dict or None, nnz list or None), plus the list
        of per-system report dicts when per_system is set."""
        L = load()
        if outs is None:
            outs = self.alloc_outputs()
        bas = (BitArray * len(outs))(*[bitarray(t, d) for t, d in zip(outs, self.dims)])
        rep = Report() if report else None
        reps = (Report * len(outs))() if (report or per_system) else None
        _check(L.pa_batch_execute(self.handle, bas, ctypes.byref(rep) if report else None, reps,
                                  _stream_ptr(stream)))
        nnz = [int(r.nnz_out) for r in reps] if reps is not None else None
        res = (outs, (rep.as_dict() if report else None), nnz if report else None)
        if per_system:
            res = res + ([_report_dict(r) for r in reps],)
        return res

    def op_times(self):
        L = load()
        cap = 4096
        ms = (ctypes.c_double * cap)()
        kd = (ctypes.c_int32 * cap)()
        mc = (ctypes.c_double * cap)()
        n = L.pa_batch_op_times(self.handle, ms, kd, mc, cap)
        if n < 0:
            _check(PA_EINVAL)
        return [(int(kd[i]), float(ms[i]), float(mc[i])) for i in range(min(n, cap))]

    def time_groups(self, reps=20, stream=None):
        return _time_groups(load().pa_batch_time_groups, self.handle, reps, stream)

    def set_wait_limit(self, polls):
        """As Plan.set_wait_limit, for the batch's single persistent launch."""
        _check(load().pa_batch_set_wait_limit(self.handle, int(polls)))

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.pa_batch_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def step_features(system, s1: int, s2: int, exposed=None) -> np.ndarray:
    """Host-only: features of the step multiplying relation sets s1 and s2 (bit masks)."""
    L = load()
    keep = _Keep()
    exposed = list(system.exposed if exposed is None else exposed)
    s = _system(keep, system)
    f = np.zeros(MODEL_FEATURES, dtype=np.float32)
    _check(L.pa_step_features(ctypes.byref(s), keep.i32(exposed), len(exposed), s1, s2,
                              f.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
    return f


def plan_step_samples(plan: "Plan"):
    """(features [k, F] float32, log2 microseconds [k]) of the last execute of a
    plan created with per_op=True, timing=2."""
    L = load()
    cap = 64
    X = np.zeros((cap, MODEL_FEATURES), dtype=np.float32)
    T = np.zeros(cap, dtype=np.float32)
    n = L.pa_plan_step_samples(plan.handle, X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                               T.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), cap)
    if n < 0:
        _check(PA_EINVAL)
    return X[:n].copy(), T[:n].copy()


class Model:
    """The learned step-time model (device-resident MLP)."""

    def __init__(self, seed: int = 0, path: Optional[str] = None):
        L = load()
        h = ctypes.c_void_p()
        if path is not None:
            _check(L.pa_model_load(os.fsencode(path), ctypes.byref(h)))
        else:
            _check(L.pa_model_create(ctypes.c_uint64(seed), ctypes.byref(h)))
        self.handle = h
        self.n_params = int(L.pa_model_n_params())

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.n_params, dtype=np.float32)
        _check(load().pa_model_get_params(self.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                          self.n_params))
        return p

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        _check(load().pa_model_set_params(self.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), p.size))

    def set_level_cost(self, us: float) -> None:
        _check(load().pa_model_set_level_cost(self.handle, float(us)))

    def forward(self, X, stream=None):
        """X: torch float32 [n, F] on the device -> torch float32 [n]."""
        import torch
        X = X.contiguous()
        Y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        _check(load().pa_model_forward(self.handle, ctypes.c_void_p(X.data_ptr()), X.shape[0],
                                       ctypes.c_void_p(Y.data_ptr()), _stream_ptr(stream)))
        return Y

    def gradient(self, X, T, stream=None):
        """(gradient torch float32 [n_params], loss) of the mean squared error."""
        import torch
        X, T = X.contiguous(), T.contiguous()
        G = torch.empty(self.n_params, dtype=torch.float32, device=X.device)
        loss = ctypes.c_float(0.0)
        _check(load().pa_model_gradient(self.handle, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                        X.shape[0], ctypes.c_void_p(G.data_ptr()), ctypes.byref(loss),
                                        _stream_ptr(stream)))
        return G, float(loss.value)

    def train_step(self, X, T, lr=1e-3, stream=None, want_loss=False):
        loss = ctypes.c_float(0.0)
        _check(load().pa_model_train_step(self.handle, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                                          X.shape[0], ctypes.c_float(lr),
                                          ctypes.byref(loss) if want_loss else None, _stream_ptr(stream)))
        return float(loss.value) if want_loss else None

    def save(self, path: str) -> None:
        _check(load().pa_model_save(self.handle, os.fsencode(path)))

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.pa_model_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def autotune(systems, reps=3, stream=None, **opts_kw):
    """Time the executor candidates for a workload (list of systems); returns
    (best dict, [tried dicts])."""
    L = load()
    keep = _Keep()
    systems = list(systems)
    arr = (System * len(systems))(*[_system(keep, s) for s in systems])
    exps = [keep.i32(list(s.exposed)) for s in systems]
    exp_ptrs = (ctypes.POINTER(ctypes.c_int32) * len(exps))(*[ctypes.cast(e, ctypes.POINTER(ctypes.c_int32)) for e in exps])
    n_exp = keep.i32([len(s.exposed) for s in systems])
    keep.items += [arr, exp_ptrs]
    opts = make_opts(keep=keep, **opts_kw)
    best = Tuning()
    cap = 32
    tried = (Tuning * cap)()
    n = ctypes.c_int32(0)
    _check(L.pa_autotune(arr, len(systems), exp_ptrs, n_exp, ctypes.byref(opts), reps, ctypes.byref(best), tried,
                         cap, ctypes.cast(ctypes.byref(n), ctypes.POINTER(ctypes.c_int32)), _stream_ptr(stream)))
    return best.as_dict(), [tried[i].as_dict() for i in range(min(n.value, cap))]


def _report_dict(rep: Report) -> dict:
    d = rep.as_dict()
    d["merges"] = [int(x) for x in rep.merges[:2 * MAX_RELATIONS]]
    return d


def solve_system(system, exposed=None, order=ORDER_EXHAUSTIVE, precision=PLOT_FP32_ESCALATE, audit=False,
                 timing=False, plain=False, given=None, model=None, stream=None, **exec_opts):
    """pa_solve_system (plan, execute, destroy); returns (device words, dims,
    report dict)."""
    L = load()
    keep = _Keep()
    exposed = list(system.exposed if exposed is None else exposed)
    dims = [int(system.axes[v][2]) for v in exposed]
    s = _system(keep, system)
    opts = make_opts(order=order, precision=precision, audit=audit, timing=timing, plain=plain, given=given,
                     model=model, keep=keep, **exec_opts)
    out = empty_bits(dims)
    ba = bitarray(out, dims)
    rep = Report()
    _check(L.pa_solve_system(ctypes.byref(s), keep.i32(exposed), len(exposed), ctypes.byref(opts), ctypes.byref(ba),
                             ctypes.byref(rep), _stream_ptr(stream)))
    return out, dims, rep.as_dict()


def solve_batch(systems, order=ORDER_EXHAUSTIVE, precision=PLOT_FP32_ESCALATE, audit=False, model=None, stream=None,
                **exec_opts):
    """pa_solve_batch (batch create, execute, destroy); returns (list of device
    words, list of dims, list of per-system report dicts)."""
    L = load()
    keep = _Keep()
    systems = list(systems)
    dims = [[int(s.axes[v][2]) for v in s.exposed] for s in systems]
    arr = (System * len(systems))(*[_system(keep, s) for s in systems])
    exps = [keep.i32(list(s.exposed)) for s in systems]
    exp_ptrs = (ctypes.POINTER(ctypes.c_int32) * len(exps))(*[ctypes.cast(e, ctypes.POINTER(ctypes.c_int32)) for e in exps])
    n_exp = keep.i32([len(s.exposed) for s in systems])
    keep.items += [arr, exp_ptrs]
    opts = make_opts(order=order, precision=precision, audit=audit, model=model, keep=keep, **exec_opts)
    outs = [empty_bits(d) for d in dims]
    bas = (BitArray * len(outs))(*[bitarray(t, d) for t, d in zip(outs, dims)])
    reps = (Report * len(outs))()
    _check(L.pa_solve_batch(arr, len(systems), exp_ptrs, n_exp, ctypes.byref(opts), bas, reps, _stream_ptr(stream)))
    return outs, dims, [_report_dict(r) for r in reps]


def workspace_bytes(system, exposed=None, order=ORDER_EXHAUSTIVE, precision=PLOT_FP32_ESCALATE, given=None,
                    model=None, **exec_opts) -> int:
    """pa_workspace_bytes: device bytes a plan of this system needs (host
    planning only, no allocation).  Raises PaError on invalid input."""
    L = load()
    keep = _Keep()
    exposed = list(system.exposed if exposed is None else exposed)
    s = _system(keep, system)
    opts = make_opts(order=order, precision=precision, given=given, model=model, keep=keep, **exec_opts)
    n = int(L.pa_workspace_bytes(ctypes.byref(s), keep.i32(exposed), len(exposed), ctypes.byref(opts)))
    if n == 0:
        raise PaError(PA_EINVAL, L.pa_last_error().decode())
    return n


def popcount(t, dims) -> int:
    L = load()
    c = ctypes.c_int64(0)
    ba = bitarray(t, dims)
    _check(L.pa_popcount(ctypes.byref(ba), ctypes.byref(c), _stream_ptr()))
    return int(c.value)


def lds_read_rate(stream=None) -> float:
    """Measured LDS read rate of the current device in bytes/s (conflict-free
    16-byte reads, one 1024-thread workgroup per CU)."""
    r = ctypes.c_double(0.0)
    _check(load().pa_lds_read_rate(ctypes.byref(r), _stream_ptr(stream)))
    return float(r.value)


def tile_popcount(t, dims, tile_rows, tile_words, stream=None):
    """Set bits per tile (density map) of a device bit array: a device int32
    tensor of shape (row blocks, word blocks) holding uint32 counts."""
    import torch
    rows = 1
    for d in dims[:-1]:
        rows *= int(d)
    rw = row_words(dims[-1]) if len(dims) else 1
    tr, tw = -(-rows // tile_rows), -(-rw // tile_words)
    out = torch.zeros(max(1, tr * tw), dtype=torch.int32, device="cuda")
    ba = bitarray(t, dims)
    _check(load().pa_tile_popcount(ctypes.byref(ba), int(tile_rows), int(tile_words), ctypes.c_void_p(out.data_ptr()),
                                   _stream_ptr(stream)))
    return out[: tr * tw].reshape(tr, tw)
