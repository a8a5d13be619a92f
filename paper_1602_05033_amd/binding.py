"""ctypes binding of liblyap.so (the C ABI in include/lyap.h).

Argument marshalling only: device memory comes from PyTorch tensors and every
step of the solver runs in the library's HIP kernels.  There is no fallback —
if the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblyap.so")

# status codes (lyap_status)
OK, NOT_CONVERGED = 0, 1
E_ARG, E_BREAKDOWN, E_INDEFINITE, E_NUMERIC, E_INNER, E_NOMEM, E_DEVICE, E_UNSUPPORTED = range(-1, -9, -1)
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", -1: "E_ARG", -2: "E_BREAKDOWN", -3: "E_INDEFINITE",
                -4: "E_NUMERIC", -5: "E_INNER", -6: "E_NOMEM", -7: "E_DEVICE", -8: "E_UNSUPPORTED"}

OP_CSR, OP_STENCIL5, OP_STENCIL7 = 0, 1, 2
STORE_F64, STORE_F32 = 0, 1
METHOD_STD, METHOD_EXT = 0, 1
PC_NONE, PC_JACOBI, PC_IC0, PC_LEARNED = 0, 1, 2, 3
K_COUNT = 16   # LYAP_K_COUNT: per-kind arrays of the results

ALLOC_FN = ct.CFUNCTYPE(ct.c_void_p, ct.c_size_t, ct.c_void_p)
FREE_FN = ct.CFUNCTYPE(None, ct.c_void_p, ct.c_void_p)


class LyapOp(ct.Structure):
    _fields_ = [("kind", ct.c_int32), ("nx", ct.c_int32), ("ny", ct.c_int32), ("nz", ct.c_int32),
                ("n", ct.c_int64), ("cc", ct.c_double), ("co", ct.c_double),
                ("diag", ct.c_void_p), ("tx", ct.c_void_p), ("ty", ct.c_void_p), ("tz", ct.c_void_p),
                ("rowptr", ct.c_void_p), ("colind", ct.c_void_p), ("val", ct.c_void_p),
                ("nnz", ct.c_int64), ("shift", ct.c_double)]


class LyapOpts(ct.Structure):
    _fields_ = [("tol", ct.c_double), ("max_iter", ct.c_int32), ("method", ct.c_int32),
                ("check_every", ct.c_int32), ("storage", ct.c_int32), ("two_pass", ct.c_int32),
                ("trunc_eps", ct.c_double), ("inner_pc", ct.c_int32), ("inner_tol", ct.c_double),
                ("inner_max_iter", ct.c_int32), ("flush_blocks", ct.c_int32), ("stream", ct.c_void_p),
                ("alloc", ALLOC_FN), ("release", FREE_FN), ("alloc_ctx", ct.c_void_p),
                ("want_T", ct.c_int32), ("verbose", ct.c_int32), ("profile", ct.c_int32)]


class LyapResult(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("s", ct.c_int32), ("ell", ct.c_int32), ("m", ct.c_int32),
                ("t", ct.c_int32), ("n", ct.c_int64), ("Z", ct.c_void_p), ("n_hist", ct.c_int32),
                ("hist_m", ct.POINTER(ct.c_int32)), ("hist_res", ct.POINTER(ct.c_double)),
                ("beta", ct.c_double), ("res", ct.c_double), ("trunc_eps", ct.c_double),
                ("times_ms", ct.c_double * 8), ("inner_iters", ct.c_int64), ("n_inner", ct.c_int32),
                ("n_checks", ct.c_int32), ("T_band", ct.POINTER(ct.c_double)),
                ("gamma", ct.POINTER(ct.c_double)), ("tau", ct.POINTER(ct.c_double)),
                ("bytes_pass1", ct.c_int64), ("bytes_spmm", ct.c_int64), ("ms_spmm", ct.c_double),
                ("owns_Z", ct.c_int32), ("kern_ms", ct.c_double * K_COUNT), ("kern_n", ct.c_int32 * K_COUNT),
                ("kern_bytes", ct.c_double * K_COUNT)]


class SylvResult(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("m", ct.c_int32), ("t", ct.c_int32), ("s", ct.c_int32),
                ("ell", ct.c_int32), ("owns_Z", ct.c_int32), ("n1", ct.c_int64),
                ("n2", ct.c_int64), ("Z1", ct.c_void_p), ("Z2", ct.c_void_p), ("n_hist", ct.c_int32),
                ("hist_m", ct.POINTER(ct.c_int32)), ("hist_res", ct.POINTER(ct.c_double)),
                ("res", ct.c_double), ("beta1", ct.c_double), ("beta2", ct.c_double), ("trunc_eps", ct.c_double),
                ("times_ms", ct.c_double * 8), ("n_checks", ct.c_int32),
                ("T_band", ct.POINTER(ct.c_double)), ("J_band", ct.POINTER(ct.c_double)),
                ("gamma1", ct.POINTER(ct.c_double)), ("gamma2", ct.POINTER(ct.c_double)),
                ("tau", ct.POINTER(ct.c_double)), ("iota", ct.POINTER(ct.c_double)),
                ("kern_ms", ct.c_double * K_COUNT), ("kern_n", ct.c_int32 * K_COUNT), ("kern_bytes", ct.c_double * K_COUNT)]


# exported symbols declared in include/lyap.h
EXPORTS = ["lyap_opts_default", "lyap_solve", "sylv_solve", "lyap_result_free", "sylv_result_free",
           "lyap_last_error", "lyap_op_apply", "lyap_op_apply_timed", "lyap_ctri", "lyap_inner_solve",
           "lyap_solve_batched", "lyap_pcnet_init", "lyap_pcnet_apply", "lyap_pcnet_grad", "lyap_pcnet_train",
           "lyap_pcnet_fcg", "sylv_solve_small_b", "lyap_sym_eig", "lyap_solve_gen",
           "lyap_pcnet_apply_noalloc", "lyap_pcnet_schur_train", "lyap_pcnet_schur_fcg"]


class LyapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def load(path: str = LIB_PATH):
    """Load liblyap.so (built by ``paper_1602_05033_amd.build``)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1602_05033_amd.build`")
    lib = ct.CDLL(path)
    lib.lyap_opts_default.argtypes = [ct.POINTER(LyapOpts)]
    lib.lyap_opts_default.restype = None
    lib.lyap_solve.argtypes = [ct.POINTER(LyapOp), ct.c_void_p, ct.c_int32, ct.c_int64, ct.POINTER(LyapOpts),
                               ct.POINTER(LyapResult)]
    lib.lyap_solve.restype = ct.c_int
    lib.sylv_solve.argtypes = [ct.POINTER(LyapOp), ct.POINTER(LyapOp), ct.c_void_p, ct.c_int64, ct.c_void_p,
                               ct.c_int64, ct.c_int32, ct.POINTER(LyapOpts), ct.POINTER(SylvResult)]
    lib.sylv_solve.restype = ct.c_int
    lib.lyap_result_free.argtypes = [ct.POINTER(LyapResult)]
    lib.lyap_result_free.restype = None
    lib.lyap_solve_gen.argtypes = [ct.POINTER(LyapOp), ct.POINTER(LyapOp), ct.c_void_p, ct.c_int32, ct.c_int64,
                                   ct.POINTER(LyapOpts), ct.POINTER(LyapResult)]
    lib.lyap_solve_gen.restype = ct.c_int
    lib.sylv_solve_small_b.argtypes = [ct.POINTER(LyapOp), ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_void_p,
                                       ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int32, ct.POINTER(LyapOpts),
                                       ct.POINTER(SylvResult)]
    lib.sylv_solve_small_b.restype = ct.c_int
    lib.lyap_sym_eig.argtypes = [ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_int64,
                                 ct.c_void_p, ct.POINTER(ct.c_int32)]
    lib.lyap_sym_eig.restype = ct.c_int
    lib.sylv_result_free.argtypes = [ct.POINTER(SylvResult)]
    lib.sylv_result_free.restype = None
    lib.lyap_last_error.argtypes = []
    lib.lyap_last_error.restype = ct.c_char_p
    lib.lyap_op_apply.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_int32, ct.c_void_p]
    lib.lyap_op_apply.restype = ct.c_int
    lib.lyap_op_apply_timed.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_int32,
                                        ct.c_int32, ct.c_void_p, ct.POINTER(ct.c_double)]
    lib.lyap_op_apply_timed.restype = ct.c_int
    lib.lyap_ctri.argtypes = [ct.c_void_p, ct.c_int32, ct.c_int32, ct.c_void_p, ct.c_void_p,
                              ct.POINTER(ct.c_double), ct.c_void_p, ct.c_void_p]
    lib.lyap_ctri.restype = ct.c_int
    lib.lyap_inner_solve.argtypes = [ct.POINTER(LyapOp), ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int32,
                                     ct.POINTER(LyapOpts), ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]
    lib.lyap_inner_solve.restype = ct.c_int
    lib.lyap_solve_batched.argtypes = [ct.c_int32, ct.POINTER(LyapOp), ct.POINTER(ct.c_void_p),
                                       ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int64), ct.POINTER(LyapOpts),
                                       ct.c_int32, ct.POINTER(LyapResult)]
    lib.lyap_solve_batched.restype = ct.c_int
    lib.lyap_pcnet_init.argtypes = [ct.c_int32, ct.c_uint64, ct.c_double, ct.c_void_p]
    lib.lyap_pcnet_init.restype = None
    lib.lyap_pcnet_apply.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                     ct.c_void_p]
    lib.lyap_pcnet_apply.restype = ct.c_int
    lib.lyap_pcnet_apply_noalloc.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                             ct.c_void_p]
    lib.lyap_pcnet_apply_noalloc.restype = ct.c_int
    lib.lyap_pcnet_grad.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                    ct.POINTER(ct.c_double), ct.c_void_p, ct.c_void_p]
    lib.lyap_pcnet_grad.restype = ct.c_int
    lib.lyap_pcnet_train.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_int32,
                                     ct.POINTER(ct.c_void_p), ct.POINTER(ct.c_void_p), ct.c_int32, ct.c_double,
                                     ct.c_void_p, ct.c_void_p]
    lib.lyap_pcnet_train.restype = ct.c_int
    lib.lyap_pcnet_fcg.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_double,
                                   ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double), ct.c_void_p]
    lib.lyap_pcnet_fcg.restype = ct.c_int
    lib.lyap_pcnet_schur_train.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_int32,
                                           ct.c_int32, ct.c_int32, ct.c_double, ct.c_void_p,
                                           ct.POINTER(ct.c_int32), ct.c_void_p]
    lib.lyap_pcnet_schur_train.restype = ct.c_int
    lib.lyap_pcnet_schur_fcg.argtypes = [ct.POINTER(LyapOp), ct.c_int32, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                         ct.c_double, ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double),
                                         ct.c_void_p]
    lib.lyap_pcnet_schur_fcg.restype = ct.c_int
    _LIB = lib
    return lib


def _check(status: int, allow=(OK,)):
    if status not in allow:
        raise LyapError(status, load().lyap_last_error().decode())
    return status


# --------------------------------------------------------------------- operators
@dataclass
class DeviceOp:
    """A ``lyap_op`` whose arrays live in torch tensors kept alive here."""
    c: LyapOp
    keep: list = field(default_factory=list)
    n: int = 0


def device_op(op, device="cuda", as_csr: bool = False, shift: float = 0.0) -> DeviceOp:
    """Marshal a ``workloads.Operator`` into a ``lyap_op`` (device arrays)."""
    import torch
    c = LyapOp()
    c.n = op.n
    c.nx, c.ny, c.nz = op.nx, op.ny, op.nz
    c.shift = shift
    keep = []
    if as_csr or op.kind == "csr":
        rp, ci, va = op.to_csr()
        trp = torch.from_numpy(rp).to(device)
        tci = torch.from_numpy(ci).to(device)
        tva = torch.from_numpy(va).to(device)
        keep += [trp, tci, tva]
        c.kind = OP_CSR
        c.rowptr, c.colind, c.val = trp.data_ptr(), tci.data_ptr(), tva.data_ptr()
        c.nnz = int(va.shape[0])
    elif op.kind == "stencil5":
        c.kind = OP_STENCIL5
        c.cc, c.co = op.cc, op.co
    elif op.kind == "stencil7":
        c.kind = OP_STENCIL7
        arrs = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(device)
                for a in (op.diag, op.tx, op.ty, op.tz)]
        keep += arrs
        c.diag, c.tx, c.ty, c.tz = (a.data_ptr() for a in arrs)
    else:
        raise ValueError(op.kind)
    return DeviceOp(c, keep, op.n)


# --------------------------------------------------------------------- allocator
class _TorchAllocator:
    """Device allocations requested by the library are torch tensors."""

    def __init__(self, device):
        self.device = device
        self.live = {}

        def _alloc(nbytes, ctx):
            import torch
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            self.live[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, ctx):
            self.live.pop(ptr, None)

        self.alloc_cb = ALLOC_FN(_alloc)
        self.free_cb = FREE_FN(_free)

    def take(self, ptr):
        return self.live.pop(ptr, None)


@dataclass
class LyapSolution:
    status: int
    Z: object            # torch tensor (n, t) on the device, column-major storage
    m: int
    t: int
    beta: float
    res: float
    hist_m: list
    hist_res: list
    times_ms: dict
    n_checks: int
    trunc_eps: float
    T_band: Optional[np.ndarray] = None
    gamma: Optional[np.ndarray] = None
    tau: Optional[np.ndarray] = None
    bytes_pass1: int = 0
    bytes_spmm: int = 0
    inner_iters: int = 0
    n_inner: int = 0
    ell: int = 0
    kernels: dict = field(default_factory=dict)
    s: int = 0           # block width used: the numerical rank of C


TIME_KEYS = ["pass1", "checks", "final", "pass2", "inner", "train", "total", "to_tol"]


KERNEL_KINDS = ["spmm_gram", "upd_gram", "chol_gram", "chol_store", "replay", "zflush", "check", "final", "init",
                "cg_dir", "cg_upd", "ext_orth", "pcnet"]


def make_opts(tol=1e-8, max_iter=5000, method=METHOD_STD, check_every=0, storage=STORE_F64, two_pass=True,
              trunc_eps=-1.0, inner_pc=PC_JACOBI, inner_tol=1e-12, inner_max_iter=5000, want_T=False,
              verbose=False, stream=None, profile=False):
    o = LyapOpts()
    load().lyap_opts_default(ct.byref(o))
    o.tol, o.max_iter, o.method, o.check_every = tol, max_iter, method, check_every
    o.storage, o.two_pass, o.trunc_eps = storage, int(bool(two_pass)), trunc_eps
    o.inner_pc, o.inner_tol, o.inner_max_iter = inner_pc, inner_tol, inner_max_iter
    o.want_T, o.verbose, o.profile = int(bool(want_T)), int(bool(verbose)), int(bool(profile))
    if stream is not None:
        o.stream = stream
    return o


def lyap_solve(dop: DeviceOp, C, raise_on_error: bool = True, **kw) -> LyapSolution:
    """Solve A X + X A + C C^T = 0.  ``C`` is an (n, s) float64 torch tensor on
    the device; returns Z (n, t) with Z Z^T ~ X."""
    import torch
    lib = load()
    n, s = C.shape
    assert n == dop.n and C.dtype == torch.float64 and C.is_cuda
    Ccm = C.t().contiguous()                   # column-major n x s, ld = n
    alloc = _TorchAllocator(C.device)
    o = make_opts(stream=torch.cuda.current_stream(C.device).cuda_stream, **kw)
    o.alloc, o.release = alloc.alloc_cb, alloc.free_cb
    r = LyapResult()
    st = lib.lyap_solve(ct.byref(dop.c), ct.c_void_p(Ccm.data_ptr()), s, n, ct.byref(o), ct.byref(r))
    msg = lib.lyap_last_error().decode()
    try:
        if raise_on_error and st not in (OK, NOT_CONVERGED):
            raise LyapError(st, msg)
        return _solution(r, st, alloc, n, C.device, msg)
    finally:
        lib.lyap_result_free(ct.byref(r))


def lyap_solve_gen(dopA: DeviceOp, dopE: DeviceOp, C, raise_on_error: bool = True, **kw) -> LyapSolution:
    """Solve A X E + E X A + C C^T = 0 (E symmetric positive definite).  ``C``
    is an (n, s) float64 device tensor, s in {1, 2, 4}; Z (n, t), Z Z^T ~ X."""
    import torch
    lib = load()
    n, s = C.shape
    assert n == dopA.n == dopE.n and C.dtype == torch.float64 and C.is_cuda
    Ccm = C.t().contiguous()
    alloc = _TorchAllocator(C.device)
    o = make_opts(stream=torch.cuda.current_stream(C.device).cuda_stream, **kw)
    o.alloc, o.release = alloc.alloc_cb, alloc.free_cb
    r = LyapResult()
    st = lib.lyap_solve_gen(ct.byref(dopA.c), ct.byref(dopE.c), ct.c_void_p(Ccm.data_ptr()), s, n, ct.byref(o),
                            ct.byref(r))
    msg = lib.lyap_last_error().decode()
    try:
        if raise_on_error and st not in (OK, NOT_CONVERGED):
            raise LyapError(st, msg)
        return _solution(r, st, alloc, n, C.device, msg)
    finally:
        lib.lyap_result_free(ct.byref(r))


def _solution(r, st, alloc, n, device, msg) -> LyapSolution:
    import torch
    Z = None
    if r.Z:
        buf = alloc.take(r.Z)
        if r.t > 0:
            Z = buf[: 8 * n * r.t].view(torch.float64).view(r.t, n).t()
        else:
            Z = torch.zeros((n, 0), dtype=torch.float64, device=device)
    ell = r.ell
    k = ell * r.m
    sol = LyapSolution(
        status=st, Z=Z, m=r.m, t=r.t, beta=r.beta, res=r.res,
        hist_m=[r.hist_m[i] for i in range(r.n_hist)], hist_res=[r.hist_res[i] for i in range(r.n_hist)],
        times_ms={k_: r.times_ms[i] for i, k_ in enumerate(TIME_KEYS)}, n_checks=r.n_checks,
        trunc_eps=r.trunc_eps, bytes_pass1=r.bytes_pass1, bytes_spmm=r.bytes_spmm,
        inner_iters=r.inner_iters, n_inner=r.n_inner, ell=ell, s=r.s,
        kernels={name: {"ms": r.kern_ms[i], "n": r.kern_n[i], "bytes_per_launch": r.kern_bytes[i]}
                 for i, name in enumerate(KERNEL_KINDS) if r.kern_n[i] > 0})
    if r.T_band:
        sol.T_band = np.ctypeslib.as_array(r.T_band, shape=(k * (ell + 1),)).copy().reshape(k, ell + 1)
        sol.gamma = np.ctypeslib.as_array(r.gamma, shape=(ell * ell,)).copy().reshape(ell, ell, order="F")
        sol.tau = np.ctypeslib.as_array(r.tau, shape=(ell * ell,)).copy().reshape(ell, ell, order="F")
    sol.error = msg
    return sol


BATCH_GRAPHS = 4  # LYAP_BATCH_GRAPHS


def lyap_solve_batched(dops, Cs, tune: bool = False, raise_on_error: bool = True, graphs: bool = False, **kw):
    """Solve a batch of Lyapunov equations in grouped launches.  ``dops``:
    list of DeviceOp; ``Cs``: list of (n_i, s_i) float64 device tensors;
    ``graphs``: replay one captured graph per first-pass step.
    Returns (status, [LyapSolution])."""
    import torch
    lib = load()
    count = len(dops)
    assert count == len(Cs) and count > 0
    ops = (LyapOp * count)(*[d.c for d in dops])
    Ccm = [C.t().contiguous() for C in Cs]
    ptrs = (ct.c_void_p * count)(*[c.data_ptr() for c in Ccm])
    ss = (ct.c_int32 * count)(*[C.shape[1] for C in Cs])
    lds = (ct.c_int64 * count)(*[C.shape[0] for C in Cs])
    alloc = _TorchAllocator(Cs[0].device)
    o = make_opts(stream=torch.cuda.current_stream(Cs[0].device).cuda_stream, **kw)
    o.alloc, o.release = alloc.alloc_cb, alloc.free_cb
    res = (LyapResult * count)()
    # tune: False / 0 fixed tile shape, True / 1 autotuned (persistent cache), 2 re-tune
    st = lib.lyap_solve_batched(count, ops, ptrs, ss, lds, ct.byref(o), int(tune) | (BATCH_GRAPHS if graphs else 0),
                                res)
    msg = lib.lyap_last_error().decode()
    try:
        if raise_on_error and st not in (OK, NOT_CONVERGED):
            raise LyapError(st, msg)
        sols = [_solution(res[i], res[i].status, alloc, Cs[i].shape[0], Cs[i].device, msg) for i in range(count)]
        return st, sols
    finally:
        for i in range(count):
            lib.lyap_result_free(ct.byref(res[i]))


def op_apply(dop: DeviceOp, V, storage: int):
    """W = A V for a row-interleaved (n, s) block (float64 or float32 tensor)."""
    import torch
    lib = load()
    W = torch.empty_like(V)
    st = lib.lyap_op_apply(ct.byref(dop.c), storage, ct.c_void_p(V.data_ptr()), ct.c_void_p(W.data_ptr()),
                           V.shape[1], ct.c_void_p(torch.cuda.current_stream(V.device).cuda_stream))
    _check(st)
    return W


def op_apply_timed(dop: DeviceOp, V, storage: int, reps: int):
    import torch
    lib = load()
    W = torch.empty_like(V)
    ms = ct.c_double(0)
    st = lib.lyap_op_apply_timed(ct.byref(dop.c), storage, ct.c_void_p(V.data_ptr()), ct.c_void_p(W.data_ptr()),
                                 V.shape[1], reps, ct.c_void_p(torch.cuda.current_stream(V.device).cuda_stream),
                                 ct.byref(ms))
    _check(st)
    return W, ms.value


def ctri(T_band: np.ndarray, gamma: np.ndarray, tau: np.ndarray):
    """Residual norm of Proposition 1 for a host band (k, ell+1); returns (res, lam)."""
    lib = load()
    k, l1 = T_band.shape
    ell = l1 - 1
    tb = np.ascontiguousarray(T_band, dtype=np.float64)
    g = np.asfortranarray(gamma, dtype=np.float64)
    t = np.asfortranarray(tau, dtype=np.float64)
    lam = np.zeros(k)
    res = ct.c_double(0)
    st = lib.lyap_ctri(tb.ctypes.data_as(ct.c_void_p), ell, k, g.ctypes.data_as(ct.c_void_p),
                       t.ctypes.data_as(ct.c_void_p), ct.byref(res), lam.ctypes.data_as(ct.c_void_p), None)
    _check(st)
    return res.value, lam


def inner_solve(dop: DeviceOp, B, raise_on_error: bool = True, **kw):
    """X = A^{-1} B by the library's inner PCG.  ``B`` is an (n, s) float64
    torch tensor on the device; returns (X, iterations, worst true relative
    residual, status)."""
    import torch
    lib = load()
    n, s = B.shape
    assert n == dop.n and B.dtype == torch.float64 and B.is_cuda
    Bcm = B.t().contiguous()
    Xcm = torch.empty_like(Bcm)
    o = make_opts(stream=torch.cuda.current_stream(B.device).cuda_stream, **kw)
    iters = ct.c_int64(0)
    rel = ct.c_double(0.0)
    st = lib.lyap_inner_solve(ct.byref(dop.c), ct.c_void_p(Bcm.data_ptr()), n, ct.c_void_p(Xcm.data_ptr()), n, s,
                              ct.byref(o), ct.byref(iters), ct.byref(rel))
    if raise_on_error and st != OK:
        raise LyapError(st, lib.lyap_last_error().decode())
    return Xcm.t(), iters.value, rel.value, st


@dataclass
class SylvSolution:
    status: int
    Z1: object
    Z2: object
    m: int
    t: int
    beta1: float
    beta2: float
    res: float
    hist_m: list
    hist_res: list
    times_ms: dict
    n_checks: int
    trunc_eps: float
    T_band: Optional[np.ndarray] = None
    J_band: Optional[np.ndarray] = None
    gamma1: Optional[np.ndarray] = None
    gamma2: Optional[np.ndarray] = None
    tau: Optional[np.ndarray] = None
    iota: Optional[np.ndarray] = None
    kernels: dict = field(default_factory=dict)
    error: str = ""


def sylv_solve(dopA: DeviceOp, dopB: DeviceOp, C1, C2, raise_on_error: bool = True, **kw) -> SylvSolution:
    """Solve A X + X B + C1 C2^T = 0; C1 (n1, s), C2 (n2, s) float64 torch
    tensors on the device.  Returns Z1 (n1, t), Z2 (n2, t) with Z1 Z2^T ~ X."""
    import torch
    lib = load()
    n1, s = C1.shape
    n2, s2 = C2.shape
    assert s == s2 and n1 == dopA.n and n2 == dopB.n
    assert C1.dtype == torch.float64 and C2.dtype == torch.float64 and C1.is_cuda and C2.is_cuda
    C1cm = C1.t().contiguous()
    C2cm = C2.t().contiguous()
    alloc = _TorchAllocator(C1.device)
    o = make_opts(stream=torch.cuda.current_stream(C1.device).cuda_stream, **kw)
    o.alloc, o.release = alloc.alloc_cb, alloc.free_cb
    r = SylvResult()
    st = lib.sylv_solve(ct.byref(dopA.c), ct.byref(dopB.c), ct.c_void_p(C1cm.data_ptr()), n1,
                        ct.c_void_p(C2cm.data_ptr()), n2, s, ct.byref(o), ct.byref(r))
    msg = lib.lyap_last_error().decode()
    try:
        if raise_on_error and st not in (OK, NOT_CONVERGED):
            raise LyapError(st, msg)
        Z1 = Z2 = None
        if r.Z1 and r.Z2:
            b1 = alloc.take(r.Z1)
            b2 = alloc.take(r.Z2)
            if r.t > 0:
                Z1 = b1[: 8 * n1 * r.t].view(torch.float64).view(r.t, n1).t()
                Z2 = b2[: 8 * n2 * r.t].view(torch.float64).view(r.t, n2).t()
            else:
                Z1 = torch.zeros((n1, 0), dtype=torch.float64, device=C1.device)
                Z2 = torch.zeros((n2, 0), dtype=torch.float64, device=C1.device)
        ell = r.ell
        k = ell * r.m
        sol = SylvSolution(
            status=st, Z1=Z1, Z2=Z2, m=r.m, t=r.t, beta1=r.beta1, beta2=r.beta2, res=r.res,
            hist_m=[r.hist_m[i] for i in range(r.n_hist)], hist_res=[r.hist_res[i] for i in range(r.n_hist)],
            times_ms={k_: r.times_ms[i] for i, k_ in enumerate(TIME_KEYS)}, n_checks=r.n_checks,
            trunc_eps=r.trunc_eps,
            kernels={name: {"ms": r.kern_ms[i], "n": r.kern_n[i], "bytes_per_launch": r.kern_bytes[i]}
                     for i, name in enumerate(KERNEL_KINDS) if r.kern_n[i] > 0})
        if r.T_band:
            sol.T_band = np.ctypeslib.as_array(r.T_band, shape=(k * (ell + 1),)).copy().reshape(k, ell + 1)
            sol.J_band = np.ctypeslib.as_array(r.J_band, shape=(k * (ell + 1),)).copy().reshape(k, ell + 1)
            for name in ("gamma1", "gamma2", "tau", "iota"):
                setattr(sol, name, np.ctypeslib.as_array(getattr(r, name), shape=(ell * ell,)).copy()
                        .reshape(ell, ell, order="F"))
        sol.error = msg
        return sol
    finally:
        lib.sylv_result_free(ct.byref(r))


def sylv_solve_small_b(dopA: DeviceOp, B, C1, C2, raise_on_error: bool = True, **kw) -> SylvSolution:
    """Solve A X + X B + C1 C2^T = 0 with a small dense B (n2, n2) float64
    torch tensor on the device (only A is projected); C1 (n1, s), C2 (n2, s)
    float64 device tensors.  Returns Z1 (n1, t), Z2 (n2, t), Z1 Z2^T ~ X."""
    import torch
    lib = load()
    n1, s = C1.shape
    n2, s2 = C2.shape
    assert s == s2 and n1 == dopA.n and tuple(B.shape) == (n2, n2)
    for x in (B, C1, C2):
        assert x.dtype == torch.float64 and x.is_cuda
    Bcm = B.t().contiguous()
    C1cm = C1.t().contiguous()
    C2cm = C2.t().contiguous()
    alloc = _TorchAllocator(C1.device)
    o = make_opts(stream=torch.cuda.current_stream(C1.device).cuda_stream, **kw)
    o.alloc, o.release = alloc.alloc_cb, alloc.free_cb
    r = SylvResult()
    st = lib.sylv_solve_small_b(ct.byref(dopA.c), ct.c_void_p(Bcm.data_ptr()), n2, n2, ct.c_void_p(C1cm.data_ptr()),
                                n1, ct.c_void_p(C2cm.data_ptr()), n2, s, ct.byref(o), ct.byref(r))
    msg = lib.lyap_last_error().decode()
    try:
        if raise_on_error and st not in (OK, NOT_CONVERGED):
            raise LyapError(st, msg)
        Z1 = Z2 = None
        if r.Z1 and r.Z2:
            b1 = alloc.take(r.Z1)
            b2 = alloc.take(r.Z2)
            if r.t > 0:
                Z1 = b1[: 8 * n1 * r.t].view(torch.float64).view(r.t, n1).t()
                Z2 = b2[: 8 * n2 * r.t].view(torch.float64).view(r.t, n2).t()
            else:
                Z1 = torch.zeros((n1, 0), dtype=torch.float64, device=C1.device)
                Z2 = torch.zeros((n2, 0), dtype=torch.float64, device=C1.device)
        ell = r.ell
        k = ell * r.m
        sol = SylvSolution(
            status=st, Z1=Z1, Z2=Z2, m=r.m, t=r.t, beta1=r.beta1, beta2=r.beta2, res=r.res,
            hist_m=[r.hist_m[i] for i in range(r.n_hist)], hist_res=[r.hist_res[i] for i in range(r.n_hist)],
            times_ms={k_: r.times_ms[i] for i, k_ in enumerate(TIME_KEYS)}, n_checks=r.n_checks,
            trunc_eps=r.trunc_eps,
            kernels={name: {"ms": r.kern_ms[i], "n": r.kern_n[i], "bytes_per_launch": r.kern_bytes[i]}
                     for i, name in enumerate(KERNEL_KINDS) if r.kern_n[i] > 0})
        if r.T_band:
            sol.T_band = np.ctypeslib.as_array(r.T_band, shape=(k * (ell + 1),)).copy().reshape(k, ell + 1)
            for name in ("gamma1", "tau"):
                setattr(sol, name, np.ctypeslib.as_array(getattr(r, name), shape=(ell * ell,)).copy()
                        .reshape(ell, ell, order="F"))
        sol.error = msg
        return sol
    finally:
        lib.sylv_result_free(ct.byref(r))


def sym_eig(B):
    """w (ascending), P, sweeps for a symmetric (n, n) float64 device tensor."""
    import torch
    lib = load()
    n = B.shape[0]
    assert tuple(B.shape) == (n, n) and B.dtype == torch.float64 and B.is_cuda
    Bcm = B.t().contiguous()
    w = torch.empty(n, dtype=torch.float64, device=B.device)
    Pcm = torch.empty((n, n), dtype=torch.float64, device=B.device)
    sw = ct.c_int32(0)
    _check(lib.lyap_sym_eig(ct.c_void_p(Bcm.data_ptr()), n, n, ct.c_void_p(w.data_ptr()),
                            ct.c_void_p(Pcm.data_ptr()), n, _stream(B.device), ct.byref(sw)))
    return w, Pcm.t(), sw.value


# ------------------------------------------------------------------ learned preconditioner components
def pcnet_init(C: int, seed: int, scale: float) -> np.ndarray:
    """SplitMix64 initial weights (host function of the library)."""
    lib = load()
    n = C * 2 * 27 + C * C * 27
    W = np.zeros(n, dtype=np.float32)
    lib.lyap_pcnet_init(C, seed, scale, W.ctypes.data_as(ct.c_void_p))
    return W


def _stream(dev):
    import torch
    return torch.cuda.current_stream(dev).cuda_stream


def pcnet_apply(dop: DeviceOp, C: int, W: np.ndarray, r):
    import torch
    lib = load()
    Wf = np.ascontiguousarray(W, dtype=np.float32)
    z = torch.empty_like(r)
    _check(lib.lyap_pcnet_apply(ct.byref(dop.c), C, Wf.ctypes.data_as(ct.c_void_p), ct.c_void_p(r.data_ptr()),
                                ct.c_void_p(z.data_ptr()), ct.c_void_p(_stream(r.device))))
    return z


def pcnet_apply_noalloc(dop: DeviceOp, C: int, W: np.ndarray, r, z):
    """z = M r through the allocation-free entry point; z is a caller-owned
    device tensor shaped like r."""
    lib = load()
    Wf = np.ascontiguousarray(W, dtype=np.float32)
    assert z.shape == r.shape and z.dtype == r.dtype and z.device == r.device
    _check(lib.lyap_pcnet_apply_noalloc(ct.byref(dop.c), C, Wf.ctypes.data_as(ct.c_void_p),
                                        ct.c_void_p(r.data_ptr()), ct.c_void_p(z.data_ptr()),
                                        ct.c_void_p(_stream(r.device))))
    return z


def pcnet_grad(dop: DeviceOp, C: int, W: np.ndarray, r, e):
    lib = load()
    Wf = np.ascontiguousarray(W, dtype=np.float32)
    g = np.zeros(Wf.shape[0])
    L = ct.c_double(0.0)
    _check(lib.lyap_pcnet_grad(ct.byref(dop.c), C, Wf.ctypes.data_as(ct.c_void_p), ct.c_void_p(r.data_ptr()),
                               ct.c_void_p(e.data_ptr()), ct.byref(L), g.ctypes.data_as(ct.c_void_p),
                               ct.c_void_p(_stream(r.device))))
    return L.value, g


def pcnet_train(dop: DeviceOp, C: int, W: np.ndarray, rs, es, steps: int, lr: float):
    lib = load()
    Wf = np.array(W, dtype=np.float32)
    P = len(rs)
    rp = (ct.c_void_p * P)(*[r.data_ptr() for r in rs])
    ep = (ct.c_void_p * P)(*[e.data_ptr() for e in es])
    losses = np.zeros(max(steps, 1))
    _check(lib.lyap_pcnet_train(ct.byref(dop.c), C, Wf.ctypes.data_as(ct.c_void_p), P, rp, ep, steps, lr,
                                losses.ctypes.data_as(ct.c_void_p), ct.c_void_p(_stream(rs[0].device))))
    return Wf, losses[:steps]


def pcnet_fcg(dop: DeviceOp, C: int, W: np.ndarray, B, eta: float = 1e-12, max_iter: int = 5000):
    import torch
    lib = load()
    Wf = np.ascontiguousarray(W, dtype=np.float32)
    X = torch.empty_like(B)
    it = ct.c_int64(0)
    rel = ct.c_double(0.0)
    st = lib.lyap_pcnet_fcg(ct.byref(dop.c), C, Wf.ctypes.data_as(ct.c_void_p), ct.c_void_p(B.data_ptr()),
                            ct.c_void_p(X.data_ptr()), eta, max_iter, ct.byref(it), ct.byref(rel),
                            ct.c_void_p(_stream(B.device)))
    return X, it.value, rel.value, st


def pcnet_schur_train(dop: DeviceOp, C: int, W: np.ndarray, b, every: int, keep: int, steps: int, lr: float):
    """Harvest pairs from the condensed IC(0) solve of A x = b and train the
    network on the black Schur complement; returns (W, losses, pairs used)."""
    lib = load()
    Wf = np.array(W, dtype=np.float32)
    losses = np.zeros(max(steps, 1))
    npairs = ct.c_int32(0)
    _check(lib.lyap_pcnet_schur_train(ct.byref(dop.c), C, Wf.ctypes.data_as(ct.c_void_p), ct.c_void_p(b.data_ptr()),
                                      every, keep, steps, lr, losses.ctypes.data_as(ct.c_void_p), ct.byref(npairs),
                                      ct.c_void_p(_stream(b.device))))
    return Wf, losses[:steps], npairs.value


def pcnet_schur_fcg(dop: DeviceOp, C: int, W: np.ndarray, B, eta: float = 1e-12, max_iter: int = 5000):
    """X = A^{-1} B by flexible CG on IC(0)'s Schur complement with the network."""
    import torch
    lib = load()
    Wf = np.ascontiguousarray(W, dtype=np.float32)
    X = torch.empty_like(B)
    it = ct.c_int64(0)
    rel = ct.c_double(0.0)
    st = lib.lyap_pcnet_schur_fcg(ct.byref(dop.c), C, Wf.ctypes.data_as(ct.c_void_p), ct.c_void_p(B.data_ptr()),
                                  ct.c_void_p(X.data_ptr()), eta, max_iter, ct.byref(it), ct.byref(rel),
                                  ct.c_void_p(_stream(B.device)))
    return X, it.value, rel.value, st
