"""Thin ctypes binding of libhmv (include/hmv.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Device buffers are torch CUDA tensors (uint64 words are carried in
int64 tensors, same bits); the stream is torch's current stream unless one
is given.  Loading fails loudly when libhmv.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhmv.so")

HANKEL, TOEPLITZ, CIRCULANT = 0, 1, 2
KINDS = {"hankel": HANKEL, "toeplitz": TOEPLITZ, "circulant": CIRCULANT}
AUTO, SPLIT_FFT, NTT, KARATSUBA, SCHOOLBOOK = 0, 1, 2, 3, 4
ALGOS = {"auto": AUTO, "split_fft": SPLIT_FFT, "ntt": NTT, "karatsuba": KARATSUBA,
         "schoolbook": SCHOOLBOOK}
OK, EINVAL, ERANGE, ENOMEM, EDEVICE, EBOUND, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MAX_P, MAX_N = 40960, 16384          # HMV_MAX_P, HMV_MAX_N

_c_i64, _c_i32, _c_int, _vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_void_p

# name -> (restype, argtypes); mirrors include/hmv.h
SIGNATURES = {
    "hmv_words": (_c_i64, [_c_i32]),
    "hmv_strerror": (ctypes.c_char_p, [_c_int]),
    "hmv_last_error": (ctypes.c_char_p, []),
    "hmv_oneshot_workspace_bytes": (_c_i64, [_c_int, _c_i64, _c_i32, _c_int]),
    "hmv_hankel_matvec": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i32, _c_int, _vp, _c_i64, _vp]),
    "hmv_toeplitz_matvec": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i32, _c_int, _vp, _c_i64, _vp]),
    "hmv_circulant_matvec": (_c_int, [_vp, _vp, _vp, _c_i64, _c_i32, _c_int, _vp, _c_i64, _vp]),
    "hmv_read_status": (_c_int, [_vp, _vp, ctypes.POINTER(_c_i32), ctypes.POINTER(ctypes.c_double)]),
    "hmv_plan_bytes": (_c_i64, [_c_int, _c_i64, _c_i32, _c_int]),
    "hmv_workspace_bytes": (_c_i64, [_c_int, _c_i64, _c_i32, _c_int]),
    "hmv_plan_h": (_c_int, [ctypes.POINTER(_vp), _c_int, _vp, _c_i64, _c_i32, _c_int, _vp, _c_i64,
                            _vp, _c_i64, _vp]),
    "hmv_plan_matvec": (_c_int, [_vp, _vp, _vp, _vp, _c_i64, _vp]),
    "hmv_plan_matvec_noalloc": (_c_int, [_vp, _vp, _vp, _vp, _vp]),
    "hmv_lanczos_workspace_bytes": (_c_i64, [_vp]),
    "hmv_lanczos": (_c_int, [_vp, _vp, _c_i32, _vp, _vp, _vp, _vp, _vp, _c_i64, _vp]),
    "hmv_fplan_bytes": (_c_i64, [_c_int, _c_i64, _c_i32, _c_i32]),
    "hmv_fplan_workspace_bytes": (_c_i64, [_c_int, _c_i64, _c_i32, _c_i32]),
    "hmv_fplan_h": (_c_int, [ctypes.POINTER(_vp), _c_int, _vp, _vp, _c_i64, _c_i32, _c_i32, _vp,
                             _c_i64, _vp, _c_i64, _vp]),
    "hmv_fplan_matvec": (_c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _c_i64, _vp]),
    "hmv_fplan_info": (_c_int, [_vp, _vp, ctypes.POINTER(_c_i32), ctypes.POINTER(_c_i32)]),
    "hmv_fplan_destroy": (_c_int, [_vp]),
    "hmv_plan_multi_workspace_bytes": (_c_i64, [_vp, _c_i32]),
    "hmv_plan_matvec_multi": (_c_int, [_vp, _c_i32, _vp, _vp, _vp, _c_i64, _vp,
                                       ctypes.POINTER(_vp)]),
    "hmv_debug_force_variants": (_c_int, [_c_i32, _c_i32]),
    "hmv_debug_force_layout": (_c_int, [_c_i32, _c_i32]),
    "hmv_debug_force_tiles": (_c_int, [_c_i32, _c_i32]),
    "hmv_batch_launches": (_c_i32, [_vp, _c_i32]),
    "hmv_autotune": (_c_int, [_c_i32]),
    "hmv_plan_workspace_bytes": (_c_i64, [_vp]),
    "hmv_plan_matvec_events": (_c_int, [_vp, _vp, _vp, _vp, _c_i64, _vp, ctypes.POINTER(_vp)]),
    "hmv_plan_info": (_c_int, [_vp, _vp]),
    "hmv_plan_destroy": (_c_int, [_vp]),
    "hmv_fft_error_bound": (ctypes.c_double, [ctypes.c_double, ctypes.c_double, _c_i32, ctypes.c_double]),
    "hmv_twiddle_beta": (ctypes.c_double, []),
    "hmv_debug_force_width": (_c_int, [_c_i32]),
    "hmv_debug_batch_spin_limit": (_c_int, [_c_i32]),
    "hmv_batch_workspace_bytes": (_c_i64, [_vp, _c_i32]),
    "hmv_batch_matvec": (_c_int, [_vp, _c_i32, _vp, _c_i64, _vp]),
    "hmv_batch_matvec_single": (_c_int, [_vp, _c_i32, _vp, _c_i64, _vp]),
    "hmv_batch_single_workspace_bytes": (_c_i64, [_vp, _c_i32]),
    "hmv_server_create": (_c_int, [ctypes.POINTER(_vp), _vp, _c_i64, _c_i32]),
    "hmv_server_add_plan": (_c_int, [_vp, _vp, ctypes.POINTER(_c_i32)]),
    "hmv_server_submit": (_c_int, [_vp, _c_i32, _c_i64, _vp, _vp, _vp, ctypes.POINTER(_c_i64)]),
    "hmv_server_poll": (_c_int, [_vp, ctypes.POINTER(_c_i64), ctypes.POINTER(_c_i32), _c_i32,
                                 ctypes.POINTER(_c_i32)]),
    "hmv_server_stats": (_c_int, [_vp, _vp]),
    "hmv_debug_force_school": (_c_int, [_c_i32]),
    "hmv_server_set_policy": (_c_int, [_vp, _c_i64, _c_i32]),
    "hmv_server_destroy": (_c_int, [_vp]),
}


class ServerStats(ctypes.Structure):
    """Mirror of hmv_server_stats_t."""
    _fields_ = [(f, ctypes.c_int64) for f in ("in_flight", "waiting", "admitted", "completed",
                                              "max_in_flight", "pool_used", "pool_peak",
                                              "pool_bytes", "large_in_flight",
                                              "max_large_in_flight", "large_bytes",
                                              "max_large")]


class Problem(ctypes.Structure):
    """Mirror of hmv_problem."""
    _fields_ = [("kind", ctypes.c_int32), ("P", ctypes.c_int32), ("n", ctypes.c_int64),
                ("h", ctypes.c_void_p), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class PlanInfo(ctypes.Structure):
    """Mirror of hmv_plan_info_t."""
    _fields_ = [("kind", ctypes.c_int32), ("algo", ctypes.c_int32), ("n", ctypes.c_int64),
                ("P", ctypes.c_int32), ("w", ctypes.c_int32), ("L", ctypes.c_int32),
                ("Nt", ctypes.c_int64), ("Nz", ctypes.c_int64), ("bound", ctypes.c_double),
                ("beta", ctypes.c_double), ("norm_h", ctypes.c_double),
                ("plan_bytes", ctypes.c_int64), ("matvec_workspace_bytes", ctypes.c_int64),
                ("cols_variant", ctypes.c_int32), ("rows_inv_variant", ctypes.c_int32),
                ("spectrum_cols", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("x_tile", ctypes.c_int32), ("y_tile", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}

_lib = None


class HmvError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = lib().hmv_strerror(code).decode() if _lib is not None else str(code)
        if code == EDEVICE and _lib is not None:
            msg += " [" + lib().hmv_last_error().decode() + "]"
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


def lib():
    """Load libhmv.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libhmv.so not built at {LIB_PATH}; run "
                              "`python -m paper_1402_5287_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(code: int, what: str = "") -> int:
    if code != OK:
        raise HmvError(code, what)
    return code


def words(P: int) -> int:
    w = lib().hmv_words(P)
    if w < 0:
        raise HmvError(int(w), "hmv_words")
    return int(w)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def to_device(words_np: np.ndarray, device="cuda"):
    """uint64 numpy words -> int64 CUDA tensor with the same bits."""
    import torch
    a = np.ascontiguousarray(words_np, dtype=np.uint64)
    return torch.from_numpy(a.view(np.int64)).to(device)


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


def workspace(nbytes: int, device="cuda"):
    import torch
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def oneshot_workspace_bytes(kind, n: int, P: int, algo="auto") -> int:
    k = KINDS.get(kind, kind)
    a = ALGOS.get(algo, algo)
    b = lib().hmv_oneshot_workspace_bytes(k, n, P, a)
    if b < 0:
        raise HmvError(int(b), "hmv_oneshot_workspace_bytes")
    return int(b)


def matvec(kind, h, x, y, n: int, P: int, algo="auto", ws=None, stream=None, check=True) -> int:
    """One-shot y = A x on device tensors.  Returns the status code."""
    k = KINDS.get(kind, kind)
    a = ALGOS.get(algo, algo)
    if ws is None:
        ws = workspace(oneshot_workspace_bytes(k, n, P, a), device=y.device)
    fn = {HANKEL: lib().hmv_hankel_matvec, TOEPLITZ: lib().hmv_toeplitz_matvec,
          CIRCULANT: lib().hmv_circulant_matvec}[k]
    rc = fn(_ptr(h), _ptr(x), _ptr(y), n, P, a, _ptr(ws), ws.numel(), _stream(stream))
    if check:
        _check(rc, "matvec")
    return rc


def read_status(ws, stream=None):
    """(status, flags, max_round_err) of the last call that used ws."""
    fl = _c_i32(0)
    err = ctypes.c_double(0.0)
    rc = lib().hmv_read_status(_ptr(ws), _stream(stream), ctypes.byref(fl), ctypes.byref(err))
    return rc, int(fl.value), float(err.value)


class Plan:
    """A resident transform of h (hmv_plan_h) plus its own plan memory.

    matvec(x, y) runs the planned product on device tensors; ws is a per-call
    scratch buffer (reused across calls on one stream)."""

    def __init__(self, kind, h, n: int, P: int, algo="auto", stream=None):
        import torch
        self.kind = KINDS.get(kind, kind)
        self.algo = ALGOS.get(algo, algo)
        self.n, self.P = int(n), int(P)
        dev = h.device
        pb = lib().hmv_plan_bytes(self.kind, n, P, self.algo)
        wb = lib().hmv_workspace_bytes(self.kind, n, P, self.algo)
        if pb < 0 or wb < 0:
            raise HmvError(int(min(pb, wb)), "plan sizes")
        self.mem = torch.empty(int(pb), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(int(wb), dtype=torch.uint8, device=dev)
        handle = ctypes.c_void_p(0)
        rc = lib().hmv_plan_h(ctypes.byref(handle), self.kind, _ptr(h), n, P, self.algo,
                              _ptr(self.mem), self.mem.numel(), _ptr(self.ws), self.ws.numel(),
                              _stream(stream))
        _check(rc, "plan_h")
        self.handle = handle
        self.mv_ws_bytes = int(lib().hmv_plan_workspace_bytes(self.handle))

    def info(self) -> dict:
        inf = PlanInfo()
        _check(lib().hmv_plan_info(self.handle, ctypes.byref(inf)), "plan_info")
        return inf.as_dict()

    def new_workspace(self):
        return workspace(self.mv_ws_bytes, device=self.mem.device)

    def matvec(self, x, y, ws=None, stream=None, check=True) -> int:
        ws = self.ws if ws is None else ws
        rc = lib().hmv_plan_matvec(self.handle, _ptr(x), _ptr(y), _ptr(ws), ws.numel(),
                                   _stream(stream))
        if check:
            _check(rc, "plan_matvec")
        return rc

    def lanczos(self, q1, steps: int, basis: bool = False, stream=None):
        """Lanczos tridiagonalisation from q1 (device words): returns device
        tensors (alpha, beta, steps_done, basis or None, ws); see hmv_lanczos."""
        import torch
        W = words(self.P)
        dev = self.mem.device
        alpha = torch.zeros((steps, W), dtype=torch.int64, device=dev)
        beta = torch.zeros((steps, W), dtype=torch.int64, device=dev)
        done = torch.zeros(1, dtype=torch.int32, device=dev)
        bas = torch.zeros((steps, self.n, W), dtype=torch.int64, device=dev) if basis else None
        nb = lib().hmv_lanczos_workspace_bytes(self.handle)
        if nb < 0:
            raise HmvError(int(nb), "hmv_lanczos_workspace_bytes")
        ws = workspace(int(nb), device=dev)
        _check(lib().hmv_lanczos(self.handle, _ptr(q1), int(steps), _ptr(alpha), _ptr(beta),
                                 _ptr(done), _ptr(bas), _ptr(ws), ws.numel(), _stream(stream)),
               "lanczos")
        return alpha, beta, done, bas, ws

    def multi_workspace(self, k: int):
        b = lib().hmv_plan_multi_workspace_bytes(self.handle, int(k))
        if b < 0:
            raise HmvError(int(b), "hmv_plan_multi_workspace_bytes")
        return workspace(int(b), device=self.mem.device)

    def matvec_multi(self, x, y, k: int, ws, events=None, stream=None, check=True) -> int:
        """Y = A [x_1 .. x_k]: x, y hold k n numbers, vector after vector."""
        arr = None
        if events is not None:
            arr = (_vp * 4)()
            for j, ev in enumerate(events):
                arr[j] = ctypes.c_void_p(ev.cuda_event) if ev is not None else None
        rc = lib().hmv_plan_matvec_multi(self.handle, int(k), _ptr(x), _ptr(y), _ptr(ws),
                                         ws.numel(), _stream(stream), arr)
        if check:
            _check(rc, "plan_matvec_multi")
        return rc

    def matvec_noalloc(self, x, y, status=None, stream=None, check=True) -> int:
        """Planned matvec on the library's fixed scratch (allocates nothing);
        status: optional 256-byte device buffer for read_status."""
        rc = lib().hmv_plan_matvec_noalloc(self.handle, _ptr(x), _ptr(y), _ptr(status),
                                           _stream(stream))
        if check:
            _check(rc, "plan_matvec_noalloc")
        return rc

    def matvec_events(self, x, y, events, ws=None, stream=None) -> int:
        """Planned matvec recording 4 torch.cuda.Event objects around its kernels."""
        ws = self.ws if ws is None else ws
        arr = (_vp * 4)()
        for k, ev in enumerate(events):
            arr[k] = ctypes.c_void_p(ev.cuda_event) if ev is not None else None
        rc = lib().hmv_plan_matvec_events(self.handle, _ptr(x), _ptr(y), _ptr(ws), ws.numel(),
                                          _stream(stream), arr)
        _check(rc, "plan_matvec_events")
        return rc

    def close(self):
        if getattr(self, "handle", None):
            lib().hmv_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FPlan:
    """Floating-point plan (hmv_fplan_h): significands as (count, W) words,
    exponents as int32 device tensors; matvec(x_sig, x_exp, y_sig, y_exp)."""

    def __init__(self, kind, h_sig, h_exp, n: int, P: int, spread: int, stream=None):
        import torch
        self.kind = KINDS.get(kind, kind)
        self.n, self.P, self.spread = int(n), int(P), int(spread)
        dev = h_sig.device
        pb = lib().hmv_fplan_bytes(self.kind, n, P, spread)
        wb = lib().hmv_fplan_workspace_bytes(self.kind, n, P, spread)
        if pb < 0 or wb < 0:
            raise HmvError(int(min(pb, wb)), "fplan sizes")
        self.mem = torch.empty(int(pb), dtype=torch.uint8, device=dev)
        self.ws = torch.empty(int(wb), dtype=torch.uint8, device=dev)
        handle = ctypes.c_void_p(0)
        rc = lib().hmv_fplan_h(ctypes.byref(handle), self.kind, _ptr(h_sig), _ptr(h_exp), n, P,
                               spread, _ptr(self.mem), self.mem.numel(), _ptr(self.ws),
                               self.ws.numel(), _stream(stream))
        _check(rc, "fplan_h")
        self.handle = handle

    def info(self) -> dict:
        inf = PlanInfo()
        Q, Eh = _c_i32(0), _c_i32(0)
        _check(lib().hmv_fplan_info(self.handle, ctypes.byref(inf), ctypes.byref(Q),
                                    ctypes.byref(Eh)), "fplan_info")
        d = inf.as_dict()
        d["Q"], d["Eh"] = int(Q.value), int(Eh.value)
        return d

    def matvec(self, x_sig, x_exp, y_sig, y_exp, ws=None, stream=None, check=True) -> int:
        ws = self.ws if ws is None else ws
        rc = lib().hmv_fplan_matvec(self.handle, _ptr(x_sig), _ptr(x_exp), _ptr(y_sig),
                                    _ptr(y_exp), _ptr(ws), ws.numel(), _stream(stream))
        if check:
            _check(rc, "fplan_matvec")
        return rc

    def close(self):
        if getattr(self, "handle", None):
            lib().hmv_fplan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(on: bool) -> None:
    """Launch-variant tuning at plan time (on by default; process-wide)."""
    _check(lib().hmv_autotune(1 if on else 0), "autotune")


def force_variants(cols: int = -1, rows_inv: int = -1) -> None:
    """Tests only: fixed split-FFT launch variants (-1, -1 = tune)."""
    _check(lib().hmv_debug_force_variants(cols, rows_inv), "force_variants")


def force_layout(z3: int = -1, pack: int = -1) -> None:
    """Tests only: split-FFT spectrum layout of later plans (z3 = 0: power-of-
    two limb transforms only; pack = 0 / 1: the two real limb bins in their
    own columns / sharing one; -1 = automatic)."""
    _check(lib().hmv_debug_force_layout(z3, pack), "force_layout")


def force_tiles(x_tile: int = -1, y_tile: int = -1) -> None:
    """Tests only: spectrum tile widths (2, 4 or 8 bins) of later split-FFT
    plans for x and y (-1 = tuned)."""
    _check(lib().hmv_debug_force_tiles(x_tile, y_tile), "force_tiles")


def force_width(w: int) -> None:
    """Tests only: restrict the binary64 limb width (0 = search)."""
    _check(lib().hmv_debug_force_width(w), "force_width")


def force_school(form: int) -> None:
    """Tests only: schoolbook form (0 vector FP64, 1 matrix-core int8, -1 default)."""
    _check(lib().hmv_debug_force_school(form), "force_school")


def batch_problems(items):
    """items: iterable of (kind, h, x, y, n, P) with device tensors."""
    arr = (Problem * len(items))()
    for k, (kind, h, x, y, n, P) in enumerate(items):
        arr[k] = Problem(KINDS.get(kind, kind), int(P), int(n), h.data_ptr(), x.data_ptr(),
                         y.data_ptr())
    return arr


def batch_workspace_bytes(problems) -> int:
    b = lib().hmv_batch_workspace_bytes(ctypes.cast(problems, ctypes.c_void_p), len(problems))
    if b < 0:
        raise HmvError(int(b), "hmv_batch_workspace_bytes")
    return int(b)


def batch_single_workspace_bytes(problems) -> int:
    b = lib().hmv_batch_single_workspace_bytes(ctypes.cast(problems, ctypes.c_void_p),
                                               len(problems))
    if b < 0:
        raise HmvError(int(b), "hmv_batch_single_workspace_bytes")
    return int(b)


def batch_launches(problems) -> int:
    n = lib().hmv_batch_launches(ctypes.cast(problems, ctypes.c_void_p), len(problems))
    if n < 0:
        raise HmvError(int(n), "hmv_batch_launches")
    return int(n)


def batch_matvec(problems, ws, stream=None, check=True) -> int:
    """All products of `problems` (from batch_problems): one launch per pass
    and transform size, each covering every instance of that size."""
    rc = lib().hmv_batch_matvec(ctypes.cast(problems, ctypes.c_void_p), len(problems), _ptr(ws),
                                ws.numel(), _stream(stream))
    if check:
        _check(rc, "batch_matvec")
    return rc


def batch_matvec_single(problems, ws, stream=None, check=True) -> int:
    """The same products in one cooperative launch (grid-wide barriers
    between the passes)."""
    rc = lib().hmv_batch_matvec_single(ctypes.cast(problems, ctypes.c_void_p), len(problems),
                                       _ptr(ws), ws.numel(), _stream(stream))
    if check:
        _check(rc, "batch_matvec_single")
    return rc


def set_batch_spin_limit(spins: int) -> None:
    """Tests only (0 = default)."""
    _check(lib().hmv_debug_batch_spin_limit(spins), "batch spin limit")


class Server:
    """Continuous-batching request scheduler (hmv_server_*) over one pool."""

    def __init__(self, pool_bytes: int, slots: int = 8, device="cuda"):
        import torch
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p(0)
        _check(lib().hmv_server_create(ctypes.byref(h), _ptr(self.pool), self.pool.numel(), slots),
               "server_create")
        self.handle = h
        self.plans = []

    def add_plan(self, plan: "Plan") -> int:
        mid = _c_i32(0)
        _check(lib().hmv_server_add_plan(self.handle, plan.handle, ctypes.byref(mid)), "add_plan")
        self.plans.append(plan)
        return int(mid.value)

    def set_policy(self, large_bytes: int, max_large: int) -> None:
        """Requests with workspace above large_bytes are large; at most
        max_large of them run at once."""
        _check(lib().hmv_server_set_policy(self.handle, int(large_bytes), int(max_large)),
               "server_set_policy")

    def submit(self, matrix_id: int, session: int, x, y, stream=None) -> int:
        """Queue one matvec; it runs after the work already queued on `stream`
        (torch's current stream by default), e.g. the kernel that wrote x."""
        rid = _c_i64(0)
        _check(lib().hmv_server_submit(self.handle, matrix_id, session, _ptr(x), _ptr(y),
                                       _stream(stream), ctypes.byref(rid)), "submit")
        return int(rid.value)

    def poll(self, cap: int = 64):
        ids = (_c_i64 * cap)()
        sts = (_c_i32 * cap)()
        nd = _c_i32(0)
        _check(lib().hmv_server_poll(self.handle, ids, sts, cap, ctypes.byref(nd)), "poll")
        return [(int(ids[k]), int(sts[k])) for k in range(nd.value)]

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().hmv_server_stats(self.handle, ctypes.byref(st)), "stats")
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().hmv_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
