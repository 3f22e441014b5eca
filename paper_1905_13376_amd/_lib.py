"""ctypes binding of libmj (include/mj.h).

Argument marshalling only: every step of every join runs in the HIP
library.  PyTorch provides device memory and streams.  If ``libmj.so`` has
not been built this module raises on import -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmj.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libmj.so not found at {LIB_PATH}; build it with "
                      "`python paper_1905_13376_amd/build.py` (no CPU fallback exists)")

_lib = ctypes.CDLL(LIB_PATH)

MJ_OK = 0
STATUS = {0: "MJ_OK", -1: "MJ_ERR_INVALID_ARG", -2: "MJ_ERR_KEY_RANGE", -3: "MJ_ERR_WORKSPACE",
          -4: "MJ_ERR_PLAN_MISMATCH", -5: "MJ_ERR_HIP", -6: "MJ_ERR_OVERFLOW",
          -7: "MJ_ERR_UNSUPPORTED"}
LINEAR, TRIANGLE = 0, 1
ALGO_3WAY, ALGO_CASCADE, ALGO_STAR, ALGO_STAR_CASCADE, ALGO_ORIENTED, ALGO_SLARGE = 0, 1, 2, 3, 4, 5
PLAN_SYMMETRIC_SIMPLE = 1          # mj_plan_t.flags: R = S = T, symmetric, no duplicates or loops
PLAN_DENSE_KEYS = 2                # mj_plan_t.flags: B and C values small enough for direct-indexed tables
PLAN_NO_DENSE = 0x100              # request (fixed plans): keep the hashed tables
PLANNERS = {"analytic": 0, "learned": 1, "fixed": 2}


class MJError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)}")


class Rel(ctypes.Structure):
    _fields_ = [("col0", ctypes.c_void_p), ("col1", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("stride", ctypes.c_int64)]


class Plan(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("algo", ctypes.c_int32),
                ("log2_nb", ctypes.c_uint32), ("log2_nc", ctypes.c_uint32),
                ("log2_share", ctypes.c_uint32), ("seed", ctypes.c_uint32),
                ("n_r", ctypes.c_uint64), ("n_s", ctypes.c_uint64), ("n_t", ctypes.c_uint64),
                ("a_domain", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("join2_size", ctypes.c_uint64), ("workspace_bytes", ctypes.c_uint64),
                ("est_ms_3way", ctypes.c_double), ("est_ms_cascade", ctypes.c_double),
                ("pred_log2_join2", ctypes.c_double), ("pred_log2_out", ctypes.c_double),
                ("est_ms_star", ctypes.c_double), ("est_ms_star_cascade", ctypes.c_double),
                ("b_domain", ctypes.c_uint32), ("c_domain", ctypes.c_uint32),
                ("input_fingerprint", ctypes.c_uint64), ("est_ms_slarge", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}

    def copy(self):
        p = Plan()
        ctypes.pointer(p)[0] = self
        return p


class BatchItem(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a_domain", ctypes.c_uint32),
                ("R", Rel), ("S", Rel), ("T", Rel), ("out", ctypes.c_void_p), ("plan", Plan)]


_vp, _u32, _u64, _i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
_RP = ctypes.POINTER(Rel)
_PP = ctypes.POINTER(Plan)

_SIGS = {
    "mj_ctx_create": ([_i32, ctypes.POINTER(_vp)], _i32),
    "mj_ctx_destroy": ([_vp], _i32),
    "mj_status_str": ([_i32], ctypes.c_char_p),
    "mj_plan_workspace": ([_i32, _u64, _u64, _u64], _u64),
    "mj_plan": ([_vp, _i32, _RP, _RP, _RP, _u32, _i32, _PP, _vp, _u64, _vp], _i32),
    "mj_linear3_count": ([_vp, _RP, _RP, _RP, _u32, _vp, _PP, _vp, _u64, _vp], _i32),
    "mj_triangle3_count": ([_vp, _RP, _RP, _RP, _vp, _PP, _vp, _u64, _vp], _i32),
    "mj_linear3_count_static_max_bytes": ([], _u64),
    "mj_linear3_count_static": ([_vp, _RP, _RP, _RP, _u32, _vp, _PP, _vp], _i32),
    "mj_cascade2_count": ([_vp, _i32, _RP, _RP, _RP, _u32, _vp, _PP, _vp, _u64, _vp], _i32),
    "mj_join2_size_workspace": ([_u64, _u64], _u64),
    "mj_linear3_distinct_workspace": ([_u64, _u64, _u64, _u32], _u64),
    "mj_linear3_distinct": ([_vp, _RP, _RP, _RP, _u32, _u32, _vp, _vp, _vp, _u64, _vp], _i32),
    "mj_linear3_materialize_workspace": ([_u64, _u64, _u64], _u64),
    "mj_linear3_materialize": ([_vp, _RP, _RP, _RP, _u64, _u64, _vp, _vp, _vp, _u64, _vp], _i32),
    "mj_join2_size": ([_vp, _RP, _RP, ctypes.POINTER(_u64), _vp, _u64, _vp], _i32),
    "mj_ctx_profile": ([_vp, _i32], _i32),
    "mj_mlp_param_bytes": ([], _u64),
    "mj_mlp_workspace": ([_u32], _u64),
    "mj_mlp_sync": ([_vp, _vp, _vp], _i32),
    "mj_mlp_forward": ([_vp, _vp, _vp, _u32, _vp, _vp], _i32),
    "mj_mlp_grads": ([_vp, _vp, _vp, _u32, _vp, _vp, _vp, _vp, _vp, _u64, _vp], _i32),
    "mj_mlp_adamw": ([_vp, _vp, ctypes.c_float, ctypes.c_float, _u32, _vp], _i32),
    "mj_sketch_workspace": ([_u64, _u64, _u64], _u64),
    "mj_sketch": ([_vp, _i32, _RP, _RP, _RP, _vp, _vp, _u64, _vp], _i32),
    "mj_ctx_set_planner": ([_vp, _vp], _i32),
    "mj_batch_workspace": ([ctypes.POINTER(BatchItem), _i32], _u64),
    "mj_batch_count": ([_vp, ctypes.POINTER(BatchItem), _i32, _vp, _u64, _vp], _i32),
    "mj_autotune": ([_vp, _i32, _RP, _RP, _RP, _u32, _vp, _PP, _vp, _u64,
                     ctypes.POINTER(ctypes.c_double), _vp], _i32),
    "mj_cost_model": ([_i32, ctypes.POINTER(ctypes.c_double), _i32,
                       ctypes.POINTER(ctypes.c_double)], _i32),
    "mj_slarge_buckets": ([_u64, _u64, _u64, ctypes.POINTER(_u32), ctypes.POINTER(_u32),
                           ctypes.POINTER(ctypes.c_double)], _i32),
    "mj_ctx_profile_read": ([_vp, _i32, _vp, _vp, _vp], _i32),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


COST = {"linear_tuples": 0, "cascade_tuples": 1, "linear_break_even_M": 2, "cyclic_tuples": 3,
        "cyclic_optimal_H": 4, "cyclic_min": 5, "join2_uniform": 6, "branch_hit": 7}


def cost_model(name: str, *args) -> float:
    """Evaluate one of the planner's analytic cost formulas (no GPU needed)."""
    arr = (ctypes.c_double * max(len(args), 1))(*[float(a) for a in args])
    out = ctypes.c_double()
    _check(_lib.mj_cost_model(COST[name], arr, len(args), ctypes.byref(out)), "mj_cost_model")
    return out.value


def slarge_buckets(n_r: int, n_s: int, n_t: int):
    """(log2 L_R, log2 L_T, modelled ms) of the S-largest plan (no GPU needed)."""
    lr, lt, ms = _u32(), _u32(), ctypes.c_double()
    _check(_lib.mj_slarge_buckets(n_r, n_s, n_t, ctypes.byref(lr), ctypes.byref(lt), ctypes.byref(ms)),
           "mj_slarge_buckets")
    return lr.value, lt.value, ms.value


def exported_symbols():
    return list(_SIGS)


def status_str(code: int) -> str:
    return _lib.mj_status_str(code).decode()


def _check(st, what):
    if st != MJ_OK:
        raise MJError(st, what)


def rel(t: torch.Tensor) -> Rel:
    """A relation from an ``[n, 2]`` 32-bit tensor (any element strides)."""
    if t.dim() != 2 or t.shape[1] != 2 or t.element_size() != 4:
        raise ValueError("a relation is an [n, 2] tensor of 32-bit keys")
    if t.is_cuda is False and t.numel() > 0:
        raise ValueError("relations must be on the GPU")
    base = t.data_ptr()
    return Rel(base, base + 4 * t.stride(1), t.shape[0], t.stride(0))


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """One libmj context bound to a device."""

    def __init__(self, device: int | None = None):
        h = ctypes.c_void_p()
        _check(_lib.mj_ctx_create(-1 if device is None else int(device), ctypes.byref(h)),
               "mj_ctx_create")
        self._h = h
        self._ws = None
        self._pws = None        # planning workspace (mj_plan allocates nothing)

    def close(self):
        if self._h:
            _lib.mj_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- profiling
    def profile(self, enable: bool = True):
        """Bracket every kernel launch with HIP events on its stream."""
        _check(_lib.mj_ctx_profile(self._h, 1 if enable else 0), "mj_ctx_profile")

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} since the last read (waits for
        the recorded events)."""
        import numpy as np
        cap = 256
        names = ctypes.create_string_buffer(32 * cap)
        ms = np.zeros(cap, dtype=np.float64)
        cnt = np.zeros(cap, dtype=np.int64)
        k = _lib.mj_ctx_profile_read(self._h, cap, names, ms.ctypes.data, cnt.ctypes.data)
        if k < 0:
            raise MJError(k, "mj_ctx_profile_read")
        raw = names.raw
        out = {}
        for i in range(k):
            nm = raw[32 * i:32 * (i + 1)].split(b"\0", 1)[0].decode()
            out[nm] = (float(ms[i]), int(cnt[i]))
        return out

    # ---------------------------------------------------------------- helpers
    def workspace(self, nbytes: int, device) -> torch.Tensor:
        """A cached workspace tensor of at least ``nbytes`` bytes."""
        nbytes = max(int(nbytes), 256)
        if self._ws is None or self._ws.numel() < nbytes or self._ws.device != device:
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        return self._ws

    def plan(self, kind, R, S, T, a_domain=0, planner="analytic", fixed: Plan | None = None,
             stream=None) -> Plan:
        p = fixed.copy() if fixed is not None else Plan()
        r, s, t = rel(R), rel(S), rel(T)
        need = _lib.mj_plan_workspace(kind, R.shape[0], S.shape[0], T.shape[0])
        if self._pws is None or self._pws.numel() < need or self._pws.device != R.device:
            self._pws = torch.empty(max(int(need), 256), dtype=torch.uint8, device=R.device)
        _check(_lib.mj_plan(self._h, kind, r, s, t, a_domain, PLANNERS[planner], ctypes.byref(p),
                            ctypes.c_void_p(self._pws.data_ptr()), self._pws.numel(),
                            _stream_ptr(stream)), "mj_plan")
        return p

    def linear3_count(self, R, S, T, a_domain, plan: Plan | None = None, out=None,
                      workspace=None, stream=None) -> torch.Tensor:
        """uint64 per-A counts (returned as an int64 tensor holding the bits)."""
        if plan is None:
            plan = self.plan(LINEAR, R, S, T, a_domain, stream=stream)
        if out is None:
            out = torch.empty(max(a_domain, 1), dtype=torch.int64, device=R.device)
        ws = workspace if workspace is not None else self.workspace(plan.workspace_bytes, R.device)
        _check(_lib.mj_linear3_count(self._h, rel(R), rel(S), rel(T), a_domain,
                                     ctypes.c_void_p(out.data_ptr()), ctypes.byref(plan),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     _stream_ptr(stream)), "mj_linear3_count")
        return out[:a_domain]

    def linear3_count_static(self, R, S, T, a_domain, plan: Plan, out=None, stream=None) -> torch.Tensor:
        """mj_linear3_count with the library's per-device scratch array as
        its workspace (no allocation in the call; ``out`` must be given for
        an allocation-free call)."""
        if out is None:
            out = torch.empty(max(a_domain, 1), dtype=torch.int64, device=R.device)
        _check(_lib.mj_linear3_count_static(self._h, rel(R), rel(S), rel(T), a_domain,
                                            ctypes.c_void_p(out.data_ptr()), ctypes.byref(plan),
                                            _stream_ptr(stream)), "mj_linear3_count_static")
        return out[:a_domain]

    def linear3_distinct(self, R, S, T, a_domain, seed=0x9E3779B9, sketch=None, est=None,
                         workspace=None, stream=None):
        """Flajolet-Martin sketches (int32 [a_domain, 16] holding the uint32
        bits) and estimates (float64 [a_domain]) of the D values per A."""
        if sketch is None:
            sketch = torch.empty((max(a_domain, 1), 16), dtype=torch.int32, device=R.device)
        if est is None:
            est = torch.empty(max(a_domain, 1), dtype=torch.float64, device=R.device)
        need = _lib.mj_linear3_distinct_workspace(R.shape[0], S.shape[0], T.shape[0], a_domain)
        ws = workspace if workspace is not None else self.workspace(need, R.device)
        _check(_lib.mj_linear3_distinct(self._h, rel(R), rel(S), rel(T), a_domain, seed & 0xFFFFFFFF,
                                        ctypes.c_void_p(sketch.data_ptr()), ctypes.c_void_p(est.data_ptr()),
                                        ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)),
               "mj_linear3_distinct")
        return sketch[:a_domain], est[:a_domain]

    def linear3_materialize(self, R, S, T, first=0, out=None, total=None, workspace=None, stream=None):
        """The result tuples (a, b, c, d) of R |x| S |x| T in nested-loop order
        (R's order, then the matching S tuples in S's order, then the matching
        T tuples in T's order), from position ``first``: written to ``out``
        (int32 [cap, 4]; as many rows as exist are written).  Without ``out``
        the total is read first and ``out`` is sized to hold the rest.
        Returns (out, total), ``total`` an int64 [1] device tensor."""
        if total is None:
            total = torch.empty(1, dtype=torch.int64, device=R.device)
        need = _lib.mj_linear3_materialize_workspace(R.shape[0], S.shape[0], T.shape[0])
        ws = workspace if workspace is not None else self.workspace(need, R.device)

        def call(o, cap):
            _check(_lib.mj_linear3_materialize(self._h, rel(R), rel(S), rel(T), first, cap,
                                               ctypes.c_void_p(o.data_ptr() if o is not None else 0),
                                               ctypes.c_void_p(total.data_ptr()),
                                               ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                               _stream_ptr(stream)), "mj_linear3_materialize")
        if out is None:
            call(None, 0)
            n = max(int(total.item()) - first, 0)
            out = torch.empty((max(n, 1), 4), dtype=torch.int32, device=R.device)
            if n:
                call(out, n)
            return out[:n], total
        if out.dim() != 2 or out.shape[1] != 4 or out.dtype != torch.int32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 [cap, 4] tensor")
        call(out, out.shape[0])
        return out, total

    def triangle3_count(self, R, S, T, plan: Plan | None = None, out=None, workspace=None,
                        stream=None) -> torch.Tensor:
        if plan is None:
            plan = self.plan(TRIANGLE, R, S, T, stream=stream)
        if out is None:
            out = torch.empty(1, dtype=torch.int64, device=R.device)
        ws = workspace if workspace is not None else self.workspace(plan.workspace_bytes, R.device)
        _check(_lib.mj_triangle3_count(self._h, rel(R), rel(S), rel(T),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.byref(plan),
                                       ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                       _stream_ptr(stream)), "mj_triangle3_count")
        return out

    def cascade2_count(self, kind, R, S, T, a_domain=0, plan: Plan | None = None, out=None,
                       workspace=None, stream=None) -> torch.Tensor:
        if plan is None:
            plan = self.plan(kind, R, S, T, a_domain, stream=stream)
        n_out = max(a_domain, 1) if kind == LINEAR else 1
        if out is None:
            out = torch.empty(n_out, dtype=torch.int64, device=R.device)
        ws = workspace if workspace is not None else self.workspace(plan.workspace_bytes, R.device)
        _check(_lib.mj_cascade2_count(self._h, kind, rel(R), rel(S), rel(T), a_domain,
                                      ctypes.c_void_p(out.data_ptr()), ctypes.byref(plan),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                      _stream_ptr(stream)), "mj_cascade2_count")
        return out[:a_domain] if kind == LINEAR else out

    def autotune(self, kind, R, S, T, a_domain=0, plan: Plan | None = None, out=None,
                 workspace=None, stream=None):
        """Time candidate plans on the device, keep the fastest (cached per
        size class).  Returns (plan, ms, counts)."""
        if plan is None:
            plan = self.plan(kind, R, S, T, a_domain, stream=stream)
        else:
            plan = plan.copy()
        n_out = max(a_domain, 1) if kind == LINEAR else 1
        if out is None:
            out = torch.empty(n_out, dtype=torch.int64, device=R.device)
        ws = workspace if workspace is not None else self.workspace(plan.workspace_bytes, R.device)
        ms = ctypes.c_double()
        _check(_lib.mj_autotune(self._h, kind, rel(R), rel(S), rel(T), a_domain,
                                ctypes.c_void_p(out.data_ptr()), ctypes.byref(plan),
                                ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.byref(ms),
                                _stream_ptr(stream)), "mj_autotune")
        return plan, ms.value, (out[:a_domain] if kind == LINEAR else out)

    def batch(self, joins, stream=None, plans=None):
        """Prepare a batch: `joins` is a list of (kind, R, S, T, a_domain).
        Returns a Batch whose run() launches mj_batch_count and whose
        `outs` hold the per-join uint64 results."""
        items = (BatchItem * len(joins))()
        outs = []
        for i, (kind, R, S, T, a_domain) in enumerate(joins):
            p = plans[i] if plans is not None else self.plan(kind, R, S, T, a_domain, stream=stream)
            n_out = max(a_domain, 1) if kind == LINEAR else 1
            o = torch.empty(n_out, dtype=torch.int64, device=R.device)
            outs.append(o[:a_domain] if kind == LINEAR else o)
            items[i].kind = kind
            items[i].a_domain = a_domain
            items[i].R, items[i].S, items[i].T = rel(R), rel(S), rel(T)
            items[i].out = o.data_ptr()
            items[i].plan = p
        nbytes = _lib.mj_batch_workspace(items, len(joins))
        device = joins[0][1].device if joins else "cuda"
        ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        return Batch(self, items, len(joins), ws, outs, [j[1:4] for j in joins])

    # ------------------------------------------------------- learned planner
    def sketch(self, kind, R, S, T, out=None, stream=None) -> torch.Tensor:
        """Degree-sketch features of a join (device fp32[100])."""
        if out is None:
            out = torch.empty(100, dtype=torch.float32, device=R.device)
        need = _lib.mj_sketch_workspace(R.shape[0], S.shape[0], T.shape[0])
        ws = self.workspace(need, R.device)
        _check(_lib.mj_sketch(self._h, kind, rel(R), rel(S), rel(T), ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(stream)),
               "mj_sketch")
        return out

    def set_planner(self, params):
        """Use the network in `params` (a LearnedPlanner buffer) for
        planner='learned'; None restores the analytic planner."""
        self._planner_keep = params
        _check(_lib.mj_ctx_set_planner(self._h, ctypes.c_void_p(params.data_ptr()) if params is not None
                                       else None), "mj_ctx_set_planner")

    def join2_size(self, R, S, stream=None) -> int:
        need = _lib.mj_join2_size_workspace(R.shape[0], S.shape[0])
        ws = self.workspace(need, R.device)
        out = ctypes.c_uint64()
        _check(_lib.mj_join2_size(self._h, rel(R), rel(S), ctypes.byref(out),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                  _stream_ptr(stream)), "mj_join2_size")
        return out.value


class Batch:
    """A prepared batch of joins (see Context.batch)."""

    def __init__(self, ctx, items, n, ws, outs, keep):
        self.ctx, self.items, self.n, self.ws, self.outs = ctx, items, n, ws, outs
        self._keep = keep          # the relations must outlive the batch

    def run(self, stream=None):
        _check(_lib.mj_batch_count(self.ctx._h, self.items, self.n,
                                   ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                   _stream_ptr(stream)), "mj_batch_count")
        return self.outs


def mlp_param_bytes() -> int:
    return int(_lib.mj_mlp_param_bytes())


def mlp_sync(ctx, params, stream=None):
    _check(_lib.mj_mlp_sync(ctx._h, ctypes.c_void_p(params.data_ptr()), _stream_ptr(stream)), "mj_mlp_sync")


def mlp_forward(ctx, params, X, Y, stream=None):
    _check(_lib.mj_mlp_forward(ctx._h, ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                               X.shape[0], ctypes.c_void_p(Y.data_ptr()), _stream_ptr(stream)),
           "mj_mlp_forward")


def mlp_grads(ctx, params, X, targets, plan_label, share_label, loss, workspace, stream=None):
    _check(_lib.mj_mlp_grads(ctx._h, ctypes.c_void_p(params.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                             X.shape[0], ctypes.c_void_p(targets.data_ptr()),
                             ctypes.c_void_p(plan_label.data_ptr()), ctypes.c_void_p(share_label.data_ptr()),
                             ctypes.c_void_p(loss.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                             workspace.numel(), _stream_ptr(stream)), "mj_mlp_grads")


def mlp_workspace_bytes(B: int) -> int:
    return int(_lib.mj_mlp_workspace(B))


def mlp_adamw(ctx, params, lr, wd, step, stream=None):
    _check(_lib.mj_mlp_adamw(ctx._h, ctypes.c_void_p(params.data_ptr()), float(lr), float(wd), int(step),
                             _stream_ptr(stream)), "mj_mlp_adamw")


def as_u64(t: torch.Tensor):
    """Host numpy uint64 view of a device int64 tensor holding uint64 bits."""
    return t.detach().cpu().numpy().view("uint64")
