"""skipm: sketch-preconditioned infeasible IPM for short-and-fat LPs on MI355X.

Thin Python binding of libskipm.so (the C ABI declared in include/skipm.h).
It only marshals arguments: torch CUDA tensors provide device memory and the
stream; every step of the solver runs in the library's HIP kernels.  Loading
fails loudly when the library has not been built (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from pathlib import Path

_LIB_PATH = Path(__file__).resolve().parent / "libskipm.so"

SKIPM_OK = 0
SKIPM_EINVAL = -1
SKIPM_ENOMEM = -2
SKIPM_EDEVICE = -3
SKIPM_ERANK = -4
SKIPM_ENOTCONV = -5
SKIPM_ESTALL = -6
SKIPM_ENAN = -7
STATUS_NAMES = {0: "ok", -1: "einval", -2: "enomem", -3: "edevice", -4: "erank",
                -5: "enotconv", -6: "estall", -7: "enan"}

SKIPM_DENSE = 0
SKIPM_CSR = 1
SKIPM_F64 = 0
SKIPM_F32 = 1
SKIPM_INNER_CG = 0
SKIPM_INNER_SD = 1
SKIPM_INNER_RICHARDSON = 2
SKIPM_SKETCH_COUNT = 0
SKIPM_SKETCH_GAUSSIAN = 1
SKIPM_PREC_FP64 = 0
SKIPM_PREC_MIXED = 1
SKIPM_PREC_BF16 = 2
SKIPM_TIER_FP64 = 0
SKIPM_TIER_FP32 = 1
SKIPM_TIER_BF16 = 2


class Problem(C.Structure):
    _fields_ = [("m", C.c_int64), ("n", C.c_int64), ("nnz", C.c_int64),
                ("format", C.c_int32), ("a_dtype", C.c_int32), ("a_vals", C.c_void_p),
                ("lda", C.c_int64), ("a_rowptr", C.c_void_p), ("a_colidx", C.c_void_p),
                ("b", C.c_void_p), ("c", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("sigma", C.c_double), ("gamma", C.c_double), ("tol_cg", C.c_double),
                ("eps_gap", C.c_double), ("eps_feas", C.c_double), ("guard", C.c_double),
                ("w", C.c_int32), ("s", C.c_int32), ("max_cg", C.c_int32),
                ("max_outer", C.c_int32), ("resketch", C.c_int32), ("precision", C.c_int32),
                ("seed", C.c_uint64), ("inner", C.c_int32), ("sketch", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("cg_total", C.c_int32),
                ("cg_max", C.c_int32), ("obj_p", C.c_double), ("obj_d", C.c_double),
                ("rel_gap", C.c_double), ("rp_norm", C.c_double), ("rd_norm", C.c_double),
                ("mu", C.c_double), ("demote_iter", C.c_int32), ("tier_final", C.c_int32),
                ("resketches", C.c_int32), ("shifts", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("mu", C.c_double), ("rp_norm", C.c_double), ("rd_norm", C.c_double),
                ("rel_gap", C.c_double), ("eta", C.c_double), ("alpha_max", C.c_double),
                ("alpha", C.c_double), ("f_norm", C.c_double), ("f0_norm", C.c_double),
                ("v_norm", C.c_double), ("v_resid", C.c_double), ("cg_iters", C.c_int32),
                ("v_iters", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("tier", C.c_int32), ("refine_steps", C.c_int32), ("resketches", C.c_int32),
                ("shifts", C.c_int32)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("f0_norm", C.c_double), ("f_norm", C.c_double)]


class RequestInfo(C.Structure):
    _fields_ = [("res", Result), ("state", C.c_int32), ("rc", C.c_int32),
                ("footprint", C.c_int64), ("device_bytes", C.c_int64),
                ("t_submit", C.c_double), ("t_start", C.c_double), ("t_done", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("budget", C.c_int64), ("in_use", C.c_int64), ("peak_in_use", C.c_int64),
                ("slots", C.c_int32), ("running", C.c_int32), ("queued", C.c_int32),
                ("completed", C.c_int64)]


SKIPM_REQ_QUEUED = 0
SKIPM_REQ_RUNNING = 1
SKIPM_REQ_DONE = 2

# every symbol the header declares, with its ctypes signature
_VP = C.c_void_p
SIGNATURES = {
    "skipm_params_default": (C.c_int, [C.POINTER(Params)]),
    "lp_create": (C.c_int, [C.POINTER(_VP), C.POINTER(Problem), C.POINTER(Params), _VP]),
    "lp_destroy": (C.c_int, [_VP]),
    "lp_reset": (C.c_int, [_VP, _VP]),
    "lp_set_iterate": (C.c_int, [_VP, _VP, _VP, _VP, C.c_int32, _VP]),
    "lp_get_iterate": (C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    "lp_get_direction": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "lp_get_residuals": (C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "sketch_hash": (C.c_int, [C.c_uint64, C.c_int64, C.c_int32, C.c_int64, C.c_int32, _VP, _VP,
                              _VP]),
    "sketch_apply": (C.c_int, [_VP, _VP, C.c_int64, _VP, C.c_int32, _VP]),
    "pcg_solve": (C.c_int, [_VP, _VP, _VP, C.c_int64, _VP, C.c_double, C.c_int32,
                            C.POINTER(PcgInfo), _VP]),
    "normal_matvec": (C.c_int, [_VP, _VP, _VP, C.c_int32, _VP]),
    "normal_matvec_timed": (C.c_int, [_VP, _VP, _VP, C.c_int32, C.POINTER(C.c_float), _VP]),
    "normal_matvec_noalloc": (C.c_int, [_VP, C.c_int32, C.c_int64, C.c_int64, C.c_int64, _VP, _VP,
                                        _VP, _VP]),
    "ipm_step": (C.c_int, [_VP, C.POINTER(StepInfo), _VP]),
    "lp_solve": (C.c_int, [_VP, C.POINTER(Result), _VP]),
    "lp_footprint": (C.c_int, [C.POINTER(Problem), C.POINTER(Params), C.POINTER(C.c_int64)]),
    "lp_device_bytes": (C.c_int, [_VP, C.POINTER(C.c_int64)]),
    "lp_kernel_timing": (C.c_int, [_VP, C.c_int32]),
    "lp_kernel_time": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "lp_sketch_time": (C.c_int, [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "lp_kernel_time_tier": (C.c_int, [_VP, C.c_int32, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64)]),
    "lp_solve_batch": (C.c_int, [C.POINTER(_VP), C.c_int32, C.POINTER(Result), C.c_int32]),
    "srv_create": (C.c_int, [C.POINTER(_VP), C.c_int64, C.c_int32]),
    "srv_submit": (C.c_int, [_VP, C.POINTER(Problem), C.POINTER(Params), _VP, _VP,
                             C.POINTER(C.c_uint64)]),
    "srv_poll": (C.c_int, [_VP, C.c_uint64, C.POINTER(RequestInfo)]),
    "srv_wait": (C.c_int, [_VP, C.c_uint64, C.POINTER(RequestInfo)]),
    "srv_now": (C.c_int, [_VP, C.POINTER(C.c_double)]),
    "srv_stats": (C.c_int, [_VP, C.POINTER(ServerStats)]),
    "srv_destroy": (C.c_int, [_VP]),
    "skipm_last_error": (C.c_char_p, []),
}

_lib = None


def library_path() -> Path:
    return _LIB_PATH


def load() -> C.CDLL:
    """Load libskipm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_2003_08072_amd.build`")
        lib = C.CDLL(str(_LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class SkipmError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().skipm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({code}): {msg}")
        self.code = code


def _check(code: int, where: str, allow=()):
    if code != SKIPM_OK and code not in allow:
        raise SkipmError(code, where)
    return code


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def default_params(**kw) -> Params:
    p = Params()
    _check(load().skipm_params_default(C.byref(p)), "skipm_params_default")
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------------------
# C-named wrappers
# ---------------------------------------------------------------------------

def sketch_hash(seed, k, s, n, w, bucket, sign, stream=None):
    """bucket: int32 CUDA tensor (n*s), sign: int8 CUDA tensor (n*s)."""
    _check(load().sketch_hash(seed, k, s, n, w, _ptr(bucket), _ptr(sign), _stream(stream)),
           "sketch_hash")


def _as_device(a, dtype):
    import numpy as np
    import torch
    if isinstance(a, torch.Tensor):
        return a.to(device="cuda", dtype=dtype)
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def problem(A, b, c, a_dtype="f64"):
    """(Problem, tensors that must outlive its use): A, b, c on the device in the
    layout lp_create reads.  A: dense (m, n) array/tensor, handed over
    column-major; a scipy.sparse matrix, handed over as CSR (int32 indices); or a
    tuple (rowptr, colidx, values) of CSR device tensors (int32 indices)."""
    import numpy as np
    import torch
    tdt = torch.float64 if a_dtype == "f64" else torch.float32
    dt = SKIPM_F64 if a_dtype == "f64" else SKIPM_F32
    bt = _as_device(b, torch.float64).contiguous()
    ct = _as_device(c, torch.float64).contiguous()
    if isinstance(A, tuple):
        # CSR already on the device: (rowptr int32 (m+1), colidx int32 (nnz), values)
        rowptr, colidx, vals = (t.contiguous() for t in A)
        assert rowptr.dtype == torch.int32 and colidx.dtype == torch.int32
        vals = vals.to(tdt)
        m, n = bt.numel(), ct.numel()
        keep = [rowptr, colidx, vals, bt, ct]
        prob = Problem(m=m, n=n, nnz=int(colidx.numel()), format=SKIPM_CSR, a_dtype=dt,
                       a_vals=vals.data_ptr(), lda=0, a_rowptr=rowptr.data_ptr(),
                       a_colidx=colidx.data_ptr(), b=bt.data_ptr(), c=ct.data_ptr())
    elif hasattr(A, "tocsr"):
        Acsr = A.tocsr()
        Acsr.sort_indices()
        m, n = Acsr.shape
        rowptr = _as_device(np.asarray(Acsr.indptr, dtype=np.int32), torch.int32)
        colidx = _as_device(np.asarray(Acsr.indices, dtype=np.int32), torch.int32)
        vals = _as_device(np.asarray(Acsr.data), tdt).contiguous()
        keep = [rowptr, colidx, vals, bt, ct]
        prob = Problem(m=m, n=n, nnz=int(Acsr.nnz), format=SKIPM_CSR, a_dtype=dt,
                       a_vals=vals.data_ptr(), lda=0, a_rowptr=rowptr.data_ptr(),
                       a_colidx=colidx.data_ptr(), b=bt.data_ptr(), c=ct.data_ptr())
    else:
        At = _as_device(A, tdt)
        m, n = At.shape
        a_col = At.t().contiguous()          # (n, m) row-major == (m, n) column-major
        keep = [a_col, bt, ct]
        prob = Problem(m=m, n=n, nnz=0, format=SKIPM_DENSE, a_dtype=dt,
                       a_vals=a_col.data_ptr(), lda=m, a_rowptr=None, a_colidx=None,
                       b=bt.data_ptr(), c=ct.data_ptr())
    return prob, keep


def footprint(prob: Problem, **params) -> int:
    """Device bytes lp_create + lp_solve allocate for `prob` (lp_footprint)."""
    out = C.c_int64()
    prm = default_params(**params)
    _check(load().lp_footprint(C.byref(prob), C.byref(prm), C.byref(out)), "lp_footprint")
    return int(out.value)


@dataclasses.dataclass
class SolveResult:
    status: int
    iters: int
    cg_total: int
    cg_max: int
    obj_p: float
    obj_d: float
    rel_gap: float
    rp_norm: float
    rd_norm: float
    mu: float
    demote_iter: int = -1
    tier_final: int = 0
    resketches: int = 0
    shifts: int = 0

    @property
    def ok(self):
        return self.status == SKIPM_OK


class LP:
    """One LP resident on the GPU (a handle from lp_create).

    A: dense (m, n) array/tensor (row-major in Python; it is handed to the
    library column-major), or a scipy.sparse matrix (handed over as CSR).
    a_dtype: "f64" or "f32" (the precision A's values are stored in).  Keyword
    parameters override skipm_params_default()."""

    def __init__(self, A, b, c, a_dtype="f64", stream=None, **params):
        self._lib = load()
        self.stream = stream
        self.handle = None
        prob, keep = problem(A, b, c, a_dtype)
        self.m, self.n = int(prob.m), int(prob.n)
        self.params = default_params(**params)
        h = C.c_void_p()
        _check(self._lib.lp_create(C.byref(h), C.byref(prob), C.byref(self.params),
                                   _stream(stream)), "lp_create")
        self.handle = h
        self.w = self.params.w if self.params.w > 0 else 4 * self.m
        del keep

    def close(self):
        if getattr(self, "handle", None):
            self._lib.lp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the entry points ----------------------------------------------------
    def reset(self):
        _check(self._lib.lp_reset(self.handle, _stream(self.stream)), "lp_reset")

    def set_iterate(self, x, y, s, reset_origin=True):
        import torch
        xs = [_as_device(v, torch.float64).contiguous() for v in (x, y, s)]
        _check(self._lib.lp_set_iterate(self.handle, *map(_ptr, xs), int(reset_origin),
                                        _stream(self.stream)), "lp_set_iterate")

    def get_iterate(self):
        import torch
        x = torch.empty(self.n, dtype=torch.float64, device="cuda")
        y = torch.empty(self.m, dtype=torch.float64, device="cuda")
        s = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(self._lib.lp_get_iterate(self.handle, _ptr(x), _ptr(y), _ptr(s),
                                        _stream(self.stream)), "lp_get_iterate")
        return x, y, s

    def get_direction(self):
        import torch
        dx = torch.empty(self.n, dtype=torch.float64, device="cuda")
        dy = torch.empty(self.m, dtype=torch.float64, device="cuda")
        ds = torch.empty(self.n, dtype=torch.float64, device="cuda")
        v = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(self._lib.lp_get_direction(self.handle, _ptr(dx), _ptr(dy), _ptr(ds), _ptr(v),
                                          _stream(self.stream)), "lp_get_direction")
        return dx, dy, ds, v

    def get_residuals(self):
        """(r_p, r_d, p, g) of the last step (lp_get_residuals)."""
        import torch
        rp = torch.empty(self.m, dtype=torch.float64, device="cuda")
        rd = torch.empty(self.n, dtype=torch.float64, device="cuda")
        p = torch.empty(self.m, dtype=torch.float64, device="cuda")
        g = torch.empty(self.m, dtype=torch.float64, device="cuda")
        _check(self._lib.lp_get_residuals(self.handle, _ptr(rp), _ptr(rd), _ptr(p), _ptr(g),
                                          _stream(self.stream)), "lp_get_residuals")
        return rp, rd, p, g

    def sketch(self, d, k, out_dtype="f64"):
        """B = A diag(d) W_k as an (m, w) tensor of float64 ("f64") or float32 ("f32")."""
        import torch
        dd = _as_device(d, torch.float64).contiguous()
        tdt = {"f64": torch.float64, "f32": torch.float32}[out_dtype]
        B = torch.empty(self.w, self.m, dtype=tdt, device="cuda")  # column-major m x w
        _check(self._lib.sketch_apply(self.handle, _ptr(dd), int(k), _ptr(B),
                                      SKIPM_F64 if out_dtype == "f64" else SKIPM_F32,
                                      _stream(self.stream)), "sketch_apply")
        return B.t()

    def pcg(self, d2, p, k, tol=1e-5, max_it=500):
        import torch
        d2t = _as_device(d2, torch.float64).contiguous()
        pt = _as_device(p, torch.float64).contiguous()
        dy = torch.empty(self.m, dtype=torch.float64, device="cuda")
        info = PcgInfo()
        _check(self._lib.pcg_solve(self.handle, _ptr(d2t), _ptr(pt), int(k), _ptr(dy),
                                   float(tol), int(max_it), C.byref(info),
                                   _stream(self.stream)), "pcg_solve")
        return dy, info

    def normal_matvec(self, u, out=None, reps=1):
        """out = A D^2 A^T u with the current D^2; the fused pass runs `reps` times."""
        import torch
        ut = _as_device(u, torch.float64).contiguous()
        if out is None:
            out = torch.empty(self.m, dtype=torch.float64, device="cuda")
        _check(self._lib.normal_matvec(self.handle, _ptr(ut), _ptr(out), int(reps),
                                       _stream(self.stream)), "normal_matvec")
        return out

    def normal_matvec_timed(self, u, reps=50):
        """Mean duration (ms) of one fused pass, from HIP events around `reps` passes."""
        import torch
        ut = _as_device(u, torch.float64).contiguous()
        out = torch.empty(self.m, dtype=torch.float64, device="cuda")
        ms = C.c_float()
        _check(self._lib.normal_matvec_timed(self.handle, _ptr(ut), _ptr(out), int(reps),
                                             C.byref(ms), _stream(self.stream)),
               "normal_matvec_timed")
        return float(ms.value)

    def step(self) -> StepInfo:
        info = StepInfo()
        _check(self._lib.ipm_step(self.handle, C.byref(info), _stream(self.stream)), "ipm_step")
        return info

    def solve(self, raise_on_error=False) -> SolveResult:
        res = Result()
        code = self._lib.lp_solve(self.handle, C.byref(res), _stream(self.stream))
        if raise_on_error:
            _check(code, "lp_solve")
        return _result(res, code)

    def kernel_timing(self, every=8):
        """Sample the CG's normal-equation product with HIP events (0: off)."""
        _check(self._lib.lp_kernel_timing(self.handle, int(every)), "lp_kernel_timing")

    def kernel_time(self):
        """(mean ms of the sampled products, number of samples)."""
        ms, n = C.c_double(), C.c_int64()
        _check(self._lib.lp_kernel_time(self.handle, C.byref(ms), C.byref(n)), "lp_kernel_time")
        return float(ms.value), int(n.value)

    def kernel_time_tier(self, tier):
        """(mean ms, samples) of the sampled products at one precision tier."""
        ms, n = C.c_double(), C.c_int64()
        _check(self._lib.lp_kernel_time_tier(self.handle, int(tier), C.byref(ms), C.byref(n)),
               "lp_kernel_time_tier")
        return float(ms.value), int(n.value)

    def sketch_time(self):
        """(mean ms of the timed sketch products B = A D W, number of samples)."""
        ms, n = C.c_double(), C.c_int64()
        _check(self._lib.lp_sketch_time(self.handle, C.byref(ms), C.byref(n)), "lp_sketch_time")
        return float(ms.value), int(n.value)

    def device_bytes(self) -> int:
        out = C.c_int64()
        _check(self._lib.lp_device_bytes(self.handle, C.byref(out)), "lp_device_bytes")
        return int(out.value)


def _result(res: Result, status=None) -> SolveResult:
    return SolveResult(res.status if status is None else status, res.iters, res.cg_total,
                       res.cg_max, res.obj_p, res.obj_d, res.rel_gap, res.rp_norm, res.rd_norm,
                       res.mu, res.demote_iter, res.tier_final, res.resketches, res.shifts)


def solve_batch(lps, workers=0):
    """lp_solve_batch over LP objects; returns one SolveResult per LP."""
    n = len(lps)
    handles = (C.c_void_p * n)(*[lp.handle.value for lp in lps])
    res = (Result * n)()
    _check(load().lp_solve_batch(handles, n, res, int(workers)), "lp_solve_batch")
    return [_result(r) for r in res]


@dataclasses.dataclass
class RequestResult:
    result: SolveResult
    state: int
    rc: int
    footprint: int
    device_bytes: int
    t_submit: float
    t_start: float
    t_done: float

    @property
    def latency(self):
        return self.t_done - self.t_submit


class Server:
    """The request server (srv_*): FIFO admission by device-memory footprint,
    `slots` LPs in flight at once."""

    def __init__(self, hbm_budget, slots=4):
        self._lib = load()
        self.handle = None
        h = C.c_void_p()
        _check(self._lib.srv_create(C.byref(h), int(hbm_budget), int(slots)), "srv_create")
        self.handle = h
        self._keep = {}

    def submit(self, A, b, c, a_dtype="f32", want_x=False, stream=None, **params):
        import torch
        prob, keep = problem(A, b, c, a_dtype)
        prm = default_params(**params)
        x = torch.empty(int(prob.n), dtype=torch.float64, device="cuda") if want_x else None
        t = C.c_uint64()
        _check(self._lib.srv_submit(self.handle, C.byref(prob), C.byref(prm), _ptr(x),
                                    _stream(stream), C.byref(t)), "srv_submit")
        self._keep[t.value] = (keep, x)
        return t.value

    def _info(self, fn, ticket):
        info = RequestInfo()
        _check(fn(self.handle, C.c_uint64(ticket), C.byref(info)), "srv_poll/wait")
        out = RequestResult(_result(info.res), info.state, info.rc, info.footprint,
                            info.device_bytes, info.t_submit, info.t_start, info.t_done)
        return out

    def poll(self, ticket):
        return self._info(self._lib.srv_poll, ticket)

    def wait(self, ticket):
        """Wait for the request; returns (RequestResult, x or None) and drops the
        request's input buffers."""
        r = self._info(self._lib.srv_wait, ticket)
        _, x = self._keep.pop(ticket, (None, None))
        return r, x

    def now(self):
        t = C.c_double()
        _check(self._lib.srv_now(self.handle, C.byref(t)), "srv_now")
        return t.value

    def stats(self):
        s = ServerStats()
        _check(self._lib.srv_stats(self.handle, C.byref(s)), "srv_stats")
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            self._lib.srv_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
