"""ctypes binding of the gfx950 C-ABI library (libgraver.so).

Argument marshalling only: every stage of the path runs in the library's
HIP kernels.  PyTorch provides device memory and the stream.  The names
mirror include/graver.h.  Loading fails loudly when the library has not
been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgraver.so")

GRAVER_FP64, GRAVER_FP32, GRAVER_BF16 = 0, 1, 2
GRAVER_F_QUADRATIC, GRAVER_F_SEPARABLE_POLY = 1, 2
GRAVER_FORM_AUTO, GRAVER_FORM_DENSE, GRAVER_FORM_SPARSE = 0, 1, 2
(GRAVER_OK, GRAVER_E_INVALID, GRAVER_E_INFEASIBLE_START, GRAVER_E_NOT_KERNEL, GRAVER_E_OVERFLOW,
 GRAVER_E_POOL_FULL, GRAVER_E_NOMEM, GRAVER_E_DEVICE, GRAVER_E_CAPACITY, GRAVER_E_CANCELLED) = range(0, -10, -1)
STATUS = {0: "OK", -1: "E_INVALID", -2: "E_INFEASIBLE_START", -3: "E_NOT_KERNEL",
          -4: "E_OVERFLOW", -5: "E_POOL_FULL", -6: "E_NOMEM", -7: "E_DEVICE", -8: "E_CAPACITY",
          -9: "E_CANCELLED"}

EXPORTED = ["graver_ctx_create", "graver_ctx_destroy", "graver_ctx_set_stream", "graver_ctx_trim", "graver_last_error",
            "graver_status_string", "graver_kernel_basis", "graver_extract", "graver_filter",
            "graver_augment", "graver_augment_noalloc", "graver_verify", "graver_init_solutions", "graver_solve", "graver_lift_inequalities",
            "graver_extract_batch", "graver_server_create", "graver_server_submit", "graver_server_wait",
            "graver_server_poll", "graver_server_cancel", "graver_server_destroy"]


class GraverError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("d", C.c_int32),
                ("A", C.c_void_p), ("b", C.c_void_p), ("l", C.c_void_p), ("u", C.c_void_p),
                ("B", C.c_void_p), ("P", C.c_void_p)]


class ObjectiveC(C.Structure):
    _fields_ = [("kind", C.c_int32), ("degree", C.c_int32), ("Q", C.c_void_p), ("c", C.c_void_p),
                ("coef", C.c_void_p)]


class ExtractParams(C.Structure):
    _fields_ = [("n_starts", C.c_int64), ("iters", C.c_int32), ("precision", C.c_int32),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("lambda1", C.c_double), ("lambda2", C.c_double),
                ("init_mode", C.c_int32), ("t0", C.c_int32), ("polish_iters", C.c_int32),
                ("collect", C.c_int32), ("seed", C.c_uint64), ("first_start", C.c_int64),
                ("pool_capacity", C.c_int64), ("any_order", C.c_int32), ("form", C.c_int32)]


class State(C.Structure):
    _fields_ = [("z", C.c_void_p), ("m", C.c_void_p), ("v", C.c_void_p)]


class ExtractStats(C.Structure):
    _fields_ = [("start_iterations", C.c_int64), ("emit_events", C.c_int64),
                ("inbox_events", C.c_int64), ("unique", C.c_int64), ("verified", C.c_int64),
                ("out_of_range", C.c_int64), ("ms_init", C.c_double), ("ms_descent", C.c_double),
                ("ms_verify", C.c_double), ("ms_sort", C.c_double),
                ("tile_slices", C.c_int32), ("tile_blocks", C.c_int32),
                ("row_entries", C.c_int32), ("row_slots", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AugmentParams(C.Structure):
    _fields_ = [("max_steps", C.c_int64)]


class InitParams(C.Structure):
    _fields_ = [("n_starts", C.c_int64), ("iters", C.c_int32), ("init_mode", C.c_int32),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("lambda3", C.c_double), ("seed", C.c_uint64), ("first_start", C.c_int64)]


class BatchParams(C.Structure):
    _fields_ = [("autotune", C.c_int32), ("use_graph", C.c_int32)]


class BatchStats(C.Structure):
    _fields_ = [("ms_descent", C.c_double), ("launches", C.c_int32), ("replays", C.c_int32),
                ("graphs", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerParams(C.Structure):
    _fields_ = [("device", C.c_int32), ("hbm_budget", C.c_int64), ("max_batch", C.c_int32),
                ("gpu_workers", C.c_int32), ("host_threads", C.c_int32), ("autotune", C.c_int32),
                ("use_graph", C.c_int32), ("batch_window_us", C.c_int32)]


class RequestC(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("A", C.c_void_p), ("b", C.c_void_p), ("l", C.c_void_p),
                ("u", C.c_void_p), ("f_kind", C.c_int32), ("f_degree", C.c_int32), ("Q", C.c_void_p),
                ("c", C.c_void_p), ("coef", C.c_void_p), ("extract", ExtractParams), ("init", InitParams),
                ("max_steps", C.c_int64), ("lll", C.c_int32), ("x_starts", C.c_void_p), ("n_x_starts", C.c_int32)]


class ResultC(C.Structure):
    _fields_ = [("status", C.c_int), ("f_best", C.c_double), ("d", C.c_int32), ("unique", C.c_int64),
                ("filtered", C.c_int64), ("feasible_starts", C.c_int64), ("augment_steps", C.c_int64),
                ("batch_size", C.c_int32), ("reused_basis", C.c_int32), ("t_submit", C.c_double),
                ("t_ready", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveParams(C.Structure):
    _fields_ = [("extract", ExtractParams), ("init", InitParams), ("max_steps", C.c_int64),
                ("lll", C.c_int32), ("x_starts", C.c_void_p), ("n_x_starts", C.c_int32), ("reuse", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("d", C.c_int32), ("reused", C.c_int32), ("best_start", C.c_int32),
                ("unique", C.c_int64), ("filtered", C.c_int64), ("feasible_starts", C.c_int64),
                ("augment_steps", C.c_int64), ("ms_basis", C.c_double), ("ms_extract", C.c_double),
                ("ms_filter", C.c_double), ("ms_init", C.c_double), ("ms_augment", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded library (import torch first so the HIP runtime is shared)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library binds to)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        L.graver_ctx_create.argtypes = [C.POINTER(C.c_void_p), C.c_int32]
        L.graver_ctx_destroy.argtypes = [C.c_void_p]
        L.graver_ctx_destroy.restype = None
        L.graver_ctx_set_stream.argtypes = [C.c_void_p, C.c_void_p]
        L.graver_ctx_trim.argtypes = [C.c_void_p]
        L.graver_last_error.restype = C.c_char_p
        L.graver_status_string.argtypes = [C.c_int]
        L.graver_status_string.restype = C.c_char_p
        L.graver_kernel_basis.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_int32, C.c_void_p,
                                          C.POINTER(C.c_int32), C.c_void_p]
        L.graver_extract.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(ExtractParams),
                                     C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(C.c_int64),
                                     C.c_void_p]
        L.graver_filter.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_int64, C.POINTER(C.c_int64)]
        L.graver_augment.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(ObjectiveC), C.c_void_p,
                                     C.c_int64, C.c_int32, C.c_void_p, C.POINTER(AugmentParams),
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]
        L.graver_augment_noalloc.argtypes = L.graver_augment.argtypes
        L.graver_verify.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                    C.POINTER(C.c_int64)]
        L.graver_init_solutions.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(InitParams),
                                            C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.POINTER(C.c_int64)]
        L.graver_solve.argtypes = [C.c_void_p, C.POINTER(Problem), C.POINTER(ObjectiveC), C.POINTER(SolveParams),
                                   C.c_void_p, C.POINTER(C.c_double), C.POINTER(SolveStats)]
        L.graver_lift_inequalities.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                               C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.c_void_p]
        L.graver_extract_batch.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.POINTER(BatchParams), C.POINTER(BatchStats)]
        L.graver_server_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(ServerParams)]
        L.graver_server_submit.argtypes = [C.c_void_p, C.POINTER(RequestC), C.POINTER(C.c_int64)]
        L.graver_server_wait.argtypes = [C.c_void_p, C.c_int64, C.POINTER(ResultC), C.c_void_p]
        L.graver_server_poll.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int32), C.POINTER(ResultC),
                                         C.c_void_p]
        L.graver_server_cancel.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]
        L.graver_server_destroy.argtypes = [C.c_void_p]
        L.graver_server_destroy.restype = None
        for name in ("graver_ctx_create", "graver_ctx_set_stream", "graver_ctx_trim", "graver_kernel_basis",
                     "graver_extract", "graver_filter", "graver_augment", "graver_augment_noalloc",
                     "graver_verify", "graver_init_solutions",
                     "graver_solve", "graver_lift_inequalities", "graver_extract_batch",
                     "graver_server_create", "graver_server_submit", "graver_server_wait",
                     "graver_server_poll", "graver_server_cancel"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise GraverError(status, lib().graver_last_error().decode())


def kernel_basis(A: np.ndarray, lll: bool = True):
    """B (n x d int64) and P = (B^T B)^-1 B^T (d x n float64), computed on the host."""
    A = np.ascontiguousarray(A, dtype=np.int64)
    m, n = A.shape
    Bbuf = np.zeros(n * n, np.int64)
    Pbuf = np.zeros(n * n, np.float64)
    d = C.c_int32(0)
    _check(lib().graver_kernel_basis(m, n, A.ctypes.data, int(lll), Bbuf.ctypes.data, C.byref(d),
                                     Pbuf.ctypes.data))
    d = d.value
    return Bbuf[: n * d].reshape(n, d).copy(), Pbuf[: d * n].reshape(d, n).copy()


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Context:
    """A library context bound to a device and torch's current stream."""

    def __init__(self, device: int = 0):
        import torch
        h = C.c_void_p()
        _check(lib().graver_ctx_create(C.byref(h), device))
        self.h = h
        self.device = device
        self.set_stream(torch.cuda.current_stream(device))

    def set_stream(self, stream):
        _check(lib().graver_ctx_set_stream(self.h, C.c_void_p(stream.cuda_stream)))

    def trim(self):
        """graver_ctx_trim: release the context's device workspace."""
        _check(lib().graver_ctx_trim(self.h))

    def close(self):
        if self.h:
            lib().graver_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class DeviceProblem:
    """Device-resident instance tensors (torch, on the GPU)."""
    A: "object"
    b: "object"
    l: "object"
    u: "object"
    B: "object"
    P: "object" = None

    @staticmethod
    def from_numpy(A, b, l, u, B, P=None, device="cuda"):
        import torch
        t = lambda x, dt: None if x is None else torch.as_tensor(np.ascontiguousarray(x), dtype=dt, device=device)
        return DeviceProblem(t(A, torch.int64), t(b, torch.int64), t(l, torch.int64), t(u, torch.int64),
                             t(B, torch.int64), t(P, torch.float64))

    def c(self) -> Problem:
        m, n = self.A.shape
        d = 0 if self.B is None else self.B.shape[1]
        return Problem(m, n, d, _ptr(self.A), _ptr(self.b), _ptr(self.l), _ptr(self.u), _ptr(self.B),
                       _ptr(self.P))


def extract_params(n_starts, iters, precision=GRAVER_FP64, init_mode=0, seed=0, t0=0,
                   pool_capacity=1 << 20, collect=1, lr=0.003, beta1=0.9, beta2=0.999, eps=1e-8,
                   lambda1=0.85, lambda2=1.0, polish_iters=0, first_start=0, any_order=False,
                   form=0) -> ExtractParams:
    return ExtractParams(n_starts, iters, precision, lr, beta1, beta2, eps, lambda1, lambda2, init_mode,
                         t0, polish_iters, collect, seed, first_start, pool_capacity, int(any_order), int(form))


def extract(ctx: Context, prob: DeviceProblem, params: ExtractParams, state=None, keys_cap=None):
    """graver_extract.  state: optional dict of float64 device tensors z, m, v
    (N x d).  Returns (keys uint8-view int8 tensor count x n on the device,
    stats dict)."""
    import torch
    n = prob.A.shape[1]
    cap = params.pool_capacity if keys_cap is None else keys_cap
    keys = torch.empty((max(cap, 1), n), dtype=torch.int8, device=prob.A.device)
    cnt = C.c_int64(0)
    stats = ExtractStats()
    st = None
    if state is not None:
        st = State(_ptr(state.get("z")), _ptr(state.get("m")), _ptr(state.get("v")))
    pc = prob.c()
    _check(lib().graver_extract(ctx.h, C.byref(pc), C.byref(params), C.byref(st) if st else None,
                                keys.data_ptr(), cap, C.byref(cnt), C.byref(stats)))
    return keys[: cnt.value], stats.as_dict()


def filter_minimal(ctx: Context, keys, keys_cap=None):
    """graver_filter on an int8 device tensor (count x n)."""
    import torch
    count, n = keys.shape
    keys = keys.contiguous()
    cap = count if keys_cap is None else keys_cap
    out = torch.empty((max(cap, 1), n), dtype=torch.int8, device=keys.device)
    cnt = C.c_int64(0)
    _check(lib().graver_filter(ctx.h, n, keys.data_ptr() if count else None, count, out.data_ptr(), cap,
                               C.byref(cnt)))
    return out[: cnt.value]


def verify(ctx: Context, A, keys):
    """graver_verify: the number of rows g of keys (int8 device tensor
    count x n) with A g != 0; A is an int64 device tensor m x n.  Returns
    (status, n_bad) without raising on GRAVER_E_NOT_KERNEL."""
    m, n = A.shape
    keys = keys.contiguous()
    nb = C.c_int64(-1)
    st = lib().graver_verify(ctx.h, m, n, A.contiguous().data_ptr(), keys.data_ptr() if keys.shape[0] else None,
                             keys.shape[0], C.byref(nb))
    if st not in (0, -3):
        _check(st)
    return st, nb.value


def objective(kind: str, Q=None, c=None, coef=None, device="cuda"):
    """Device tensors + ObjectiveC for graver_augment."""
    import torch
    t = lambda x: None if x is None else torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=device)
    if kind == "quadratic":
        Qt, ct = t(Q), t(c)
        return (Qt, ct), ObjectiveC(GRAVER_F_QUADRATIC, 0, _ptr(Qt), _ptr(ct), None)
    cf = t(coef)
    return (cf,), ObjectiveC(GRAVER_F_SEPARABLE_POLY, int(coef.shape[1]) - 1, None, None, _ptr(cf))


def augment(ctx: Context, prob: DeviceProblem, obj, dirs, x_starts, max_steps: int = 10 ** 6, out=None,
            noalloc: bool = False):
    """graver_augment (graver_augment_noalloc with noalloc=True).  obj = the
    pair returned by objective().  out: optional (x_out, f_out, steps_out)
    device tensors to write.  Returns (x_out, f_out, steps_out) device tensors
    and the best start index."""
    import torch
    _, oc = obj
    S, n = x_starts.shape
    x_starts = x_starts.contiguous()
    dirs = dirs.contiguous()
    if out is None:
        x_out = torch.empty_like(x_starts)
        f_out = torch.empty(S, dtype=torch.float64, device=x_starts.device)
        steps = torch.empty(S, dtype=torch.int64, device=x_starts.device)
    else:
        x_out, f_out, steps = out
    best = C.c_int32(-1)
    pc = prob.c()
    prm = AugmentParams(max_steps)
    fn = lib().graver_augment_noalloc if noalloc else lib().graver_augment
    _check(fn(ctx.h, C.byref(pc), C.byref(oc), dirs.data_ptr() if dirs.shape[0] else None,
              dirs.shape[0], S, x_starts.data_ptr(), C.byref(prm), x_out.data_ptr(),
              f_out.data_ptr(), steps.data_ptr(), C.byref(best)))
    return x_out, f_out, steps, best.value


def init_params(n_starts, iters, init_mode=0, seed=0, first_start=0, lr=0.003, beta1=0.9, beta2=0.999,
                eps=1e-8, lambda3=0.1) -> InitParams:
    return InitParams(n_starts, iters, init_mode, lr, beta1, beta2, eps, lambda3, seed, first_start)


def init_solutions(ctx: Context, prob: DeviceProblem, params: InitParams, x0=None):
    """graver_init_solutions.  Returns (x_final float64 S x n, rounded int64
    S x n, feasible int32 S) device tensors and the feasible count."""
    import torch
    S = params.n_starts
    n = prob.A.shape[1]
    dev = prob.A.device
    x_out = torch.empty((S, n), dtype=torch.float64, device=dev)
    sol = torch.empty((S, n), dtype=torch.int64, device=dev)
    feas = torch.empty(S, dtype=torch.int32, device=dev)
    if x0 is not None:
        x0 = x0.contiguous()
    cnt = C.c_int64(0)
    pc = prob.c()
    _check(lib().graver_init_solutions(ctx.h, C.byref(pc), C.byref(params), _ptr(x0), x_out.data_ptr(),
                                       sol.data_ptr(), feas.data_ptr(), C.byref(cnt)))
    return x_out, sol, feas, cnt.value


def solve_params(extract: ExtractParams, init: InitParams, max_steps=10 ** 6, lll=True, reuse=True,
                 x_starts=None) -> SolveParams:
    """x_starts: optional int64 device tensor (S' x n) of feasible points;
    the caller keeps it alive for the solve call."""
    xs = None if x_starts is None else x_starts.contiguous()
    p = SolveParams(extract, init, max_steps, int(lll), _ptr(xs), 0 if xs is None else xs.shape[0], int(reuse))
    p._keep = xs
    return p


def solve(ctx: Context, prob: DeviceProblem, obj, params: SolveParams):
    """graver_solve.  prob.B / prob.P may be None (the library computes
    them).  Returns (x_best int64 device tensor, f_best, stats dict)."""
    import torch
    _, oc = obj
    n = prob.A.shape[1]
    x = torch.empty(n, dtype=torch.int64, device=prob.A.device)
    fb = C.c_double(0.0)
    stt = SolveStats()
    pc = prob.c()
    _check(lib().graver_solve(ctx.h, C.byref(pc), C.byref(oc), C.byref(params), x.data_ptr(), C.byref(fb),
                              C.byref(stt)))
    return x, fb.value, stt.as_dict()


def lift_inequalities(A, b, l, u, G, h, B=None):
    """graver_lift_inequalities on host arrays: (A', b', l', u', [B; G B])."""
    c = lambda x: np.ascontiguousarray(x, dtype=np.int64)
    A, b, l, u, G, h = c(A), c(b), c(l), c(u), c(G), c(h)
    m, n = A.shape
    mi = G.shape[0]
    A2 = np.zeros((m + mi, n + mi), np.int64)
    b2 = np.zeros(m + mi, np.int64)
    l2 = np.zeros(n + mi, np.int64)
    u2 = np.zeros(n + mi, np.int64)
    d = 0 if B is None else B.shape[1]
    Bt = None if B is None else np.zeros((n + mi, d), np.int64)
    Bc = None if B is None else c(B)
    _check(lib().graver_lift_inequalities(m, n, A.ctypes.data if m else None, b.ctypes.data if m else None,
                                          l.ctypes.data, u.ctypes.data, mi, G.ctypes.data, h.ctypes.data, d,
                                          None if Bc is None else Bc.ctypes.data, A2.ctypes.data, b2.ctypes.data,
                                          l2.ctypes.data, u2.ctypes.data, None if Bt is None else Bt.ctypes.data))
    return A2, b2, l2, u2, Bt


def extract_batch(ctx: Context, probs, params, states=None, autotune=False, use_graph=False, keys_caps=None):
    """graver_extract_batch.  probs: list of DeviceProblem; params: list of
    ExtractParams; states: optional list of state dicts (or None entries).
    Returns (list of key tensors, list of stats dicts, batch stats dict)."""
    import torch
    cnt = len(probs)
    pcs = (Problem * cnt)(*[p.c() for p in probs])
    prm = (ExtractParams * cnt)(*params)
    caps = [p.pool_capacity for p in params] if keys_caps is None else list(keys_caps)
    keys = [torch.empty((max(c, 1), pr.A.shape[1]), dtype=torch.int8, device=pr.A.device) for c, pr in zip(caps, probs)]
    kptr = (C.c_void_p * cnt)(*[k.data_ptr() for k in keys])
    kcap = (C.c_int64 * cnt)(*caps)
    out = (C.c_int64 * cnt)()
    stt = (ExtractStats * cnt)()
    st_structs = None
    st_ptrs = None
    if states is not None:
        st_structs = [None if st is None else State(_ptr(st.get("z")), _ptr(st.get("m")), _ptr(st.get("v")))
                      for st in states]
        st_ptrs = (C.c_void_p * cnt)(*[None if x is None else C.addressof(x) for x in st_structs])
    bp = BatchParams(int(autotune), int(use_graph))
    bs = BatchStats()
    _check(lib().graver_extract_batch(ctx.h, cnt, C.byref(pcs), C.byref(prm), st_ptrs, kptr, kcap, out,
                                      C.byref(stt), C.byref(bp), C.byref(bs)))
    return [k[: out[i]] for i, k in enumerate(keys)], [stt[i].as_dict() for i in range(cnt)], bs.as_dict()


class Server:
    """graver_server_*: submit host-side requests, wait for results."""

    def __init__(self, device=0, hbm_budget=64 << 30, max_batch=16, gpu_workers=2, host_threads=4,
                 autotune=False, use_graph=False, batch_window_us=0):
        lib()
        h = C.c_void_p()
        prm = ServerParams(device, hbm_budget, max_batch, gpu_workers, host_threads, int(autotune),
                           int(use_graph), batch_window_us)
        _check(lib().graver_server_create(C.byref(h), C.byref(prm)))
        self.h = h
        self.n = {}

    def submit(self, A, b, l, u, extract: ExtractParams, init: InitParams, Q=None, c=None, coef=None,
               max_steps=10 ** 6, lll=True, x_starts=None) -> int:
        a = lambda x, dt: None if x is None else np.ascontiguousarray(x, dtype=dt)
        A, b, l, u = a(A, np.int64), a(b, np.int64), a(l, np.int64), a(u, np.int64)
        Q, c, coef = a(Q, np.float64), a(c, np.float64), a(coef, np.float64)
        xs = a(x_starts, np.int64)
        m, n = A.shape
        p = lambda x: None if x is None else x.ctypes.data
        kind = GRAVER_F_QUADRATIC if coef is None else GRAVER_F_SEPARABLE_POLY
        deg = 0 if coef is None else coef.shape[1] - 1
        req = RequestC(m, n, p(A), p(b), p(l), p(u), kind, deg, p(Q), p(c), p(coef), extract, init, max_steps,
                       int(lll), p(xs), 0 if xs is None else xs.shape[0])
        t = C.c_int64(0)
        _check(lib().graver_server_submit(self.h, C.byref(req), C.byref(t)))
        self.n[t.value] = n
        return t.value

    def wait(self, ticket):
        """Returns (result dict, x_best numpy int64 or None)."""
        res = ResultC()
        n = self.n.pop(ticket)
        x = np.zeros(n, np.int64)
        _check(lib().graver_server_wait(self.h, ticket, C.byref(res), x.ctypes.data))
        r = res.as_dict()
        return r, (x if r["status"] == 0 else None)

    def poll(self, ticket):
        """(done, result dict or None, x_best or None) without blocking."""
        res = ResultC()
        n = self.n[ticket]
        x = np.zeros(n, np.int64)
        done = C.c_int32(0)
        _check(lib().graver_server_poll(self.h, ticket, C.byref(done), C.byref(res), x.ctypes.data))
        if not done.value:
            return False, None, None
        self.n.pop(ticket)
        r = res.as_dict()
        return True, r, (x if r["status"] == 0 else None)

    def cancel(self, ticket) -> bool:
        """True when the request will end with GRAVER_E_CANCELLED."""
        c = C.c_int32(0)
        _check(lib().graver_server_cancel(self.h, ticket, C.byref(c)))
        return bool(c.value)

    def close(self):
        if self.h:
            lib().graver_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
