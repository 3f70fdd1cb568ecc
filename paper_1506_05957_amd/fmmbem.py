"""ctypes binding of libfmmbem (argument marshalling only).

Every function carries the name of the C entry point it calls (see
include/fmmbem.h for the contract).  Device vectors are torch CUDA tensors of
float64; streams are torch streams (the current stream by default).  There is
no fallback: if the HIP library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loaded first so that the library shares torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmmbem.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, EBUSY, EINTERNAL = 0, -1, -2, -3, -4, -5, -6
LAPLACE, STOKES, LAPLACE_DL = 0, 1, 2  # single layer, Stokes single layer, 1/2 I - K (exterior Neumann)
FP64, FP32 = 0, 1
FIXED, RELAX_SHIFT, RELAX_BF = 0, 1, 2
P_MAX, P_MAX_FP32 = 20, 14
N_STAGES = 11
STAGES = tuple(f"{s}_{pr}" for pr in ("fp64", "fp32")
               for s in ("p2p", "m2l", "p2m_m2m", "l2l_l2p", "charges_correction")) + ("krylov",)

c_i32, c_i64, c_d, c_u8, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint8, ctypes.c_void_p
P = ctypes.POINTER


class fmmbem_mesh(ctypes.Structure):
    _fields_ = [("n_vertices", c_i64), ("n_triangles", c_i64), ("xyz", P(c_d)), ("tri", P(c_i32))]


ALLOC_FN = ctypes.CFUNCTYPE(c_vp, ctypes.c_size_t, c_vp)
FREE_FN = ctypes.CFUNCTYPE(None, c_vp, c_vp)


class fmmbem_params(ctypes.Structure):
    _fields_ = [("theta", c_d), ("ncrit", c_i32), ("p_max", c_i32), ("mu", c_d), ("near_stored", c_i32),
                ("m2l_stored", c_i32), ("quad_far", c_i32), ("quad_near", c_i32), ("near_factor", c_d),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_user", c_vp)]


class fmmbem_schedule(ctypes.Structure):
    _fields_ = [("rule", c_i32), ("p_init", c_i32), ("p_min", c_i32), ("mixed", c_i32), ("fp32_eps", c_d),
                ("restart", c_i32), ("max_iter", c_i32)]


class fmmbem_report(ctypes.Structure):
    _fields_ = [("iterations", c_i32), ("restarts", c_i32), ("converged", c_i32), ("fallbacks", c_i32),
                ("stalls", c_i32), ("p_floor", c_i32), ("rel_res_implicit", c_d), ("rel_res_true", c_d),
                ("t_solve_s", c_d), ("matvecs", c_i64),
                ("t_p2p_s", c_d), ("t_m2l_s", c_d), ("t_other_fmm_s", c_d), ("t_krylov_s", c_d),
                ("hist_cap", c_i32), ("p_hist", P(c_i32)), ("prec_hist", P(c_u8)), ("res_hist", P(c_d))]


class fmmbem_stats(ctypes.Structure):
    _fields_ = [("n_panels", c_i64), ("n_unknowns", c_i64), ("n_sources", c_i64), ("n_boxes", c_i32),
                ("n_leaves", c_i32), ("n_levels", c_i32), ("max_leaf", c_i32), ("n_m2l", c_i64),
                ("n_p2p", c_i64), ("p2p_interactions", c_i64), ("nnz_correction", c_i64),
                ("device_bytes", c_i64), ("near_entries", c_i64), ("n_translations", c_i64),
                ("m2l_op_bytes", c_i64)]


class fmmbem_server_params(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", c_i64), ("max_active", c_i32), ("n_streams", c_i32)]


class fmmbem_request_info(ctypes.Structure):
    _fields_ = [("arrival_s", c_d), ("admit_s", c_d), ("finish_s", c_d), ("iterations", c_i32),
                ("converged", c_i32), ("rel_res_true", c_d), ("device_bytes", c_i64)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("fmmbem_params_default", None, [P(fmmbem_params)])
_sig("fmmbem_schedule_default", None, [P(fmmbem_schedule), ctypes.c_int])
_sig("fmmbem_build", ctypes.c_int, [P(fmmbem_mesh), ctypes.c_int, P(fmmbem_params), c_vp, P(c_vp)])
_sig("fmmbem_matvec", ctypes.c_int, [c_vp, c_i32, c_i32, c_vp, c_vp, c_vp])
_sig("fmmbem_solve_ctx", ctypes.c_int, [c_vp, c_vp, c_d, P(fmmbem_schedule), c_vp, P(fmmbem_report), c_vp])
_sig("fmmbem_solve_ctx_static", ctypes.c_int, [c_vp, c_vp, c_d, P(fmmbem_schedule), c_vp, P(fmmbem_report), c_vp])
_sig("fmmbem_solve", ctypes.c_int, [P(fmmbem_mesh), P(c_d), ctypes.c_int, c_d, P(fmmbem_schedule),
                                    P(fmmbem_params), P(c_d), P(fmmbem_report)])
_sig("fmmbem_get_stats", ctypes.c_int, [c_vp, P(fmmbem_stats)])
_sig("fmmbem_destroy", None, [c_vp])
_sig("fmmbem_last_error", ctypes.c_char_p, [])
_sig("fmmbem_set_timing", ctypes.c_int, [c_vp, ctypes.c_int])
_sig("fmmbem_set_timing_stages", ctypes.c_int, [c_vp, ctypes.c_uint32])
_sig("fmmbem_get_timing", ctypes.c_int, [c_vp, P(c_d), P(c_i64), P(c_d), ctypes.c_int])
_sig("fmmbem_tree_sizes", ctypes.c_int, [c_vp, P(c_i64)])
_sig("fmmbem_tree_get", ctypes.c_int, [c_vp, P(c_i32), P(ctypes.c_uint64), P(c_i32), P(c_d), P(c_i32),
                                       P(c_i32), P(c_d)])
_sig("fmmbem_server_create", ctypes.c_int, [P(fmmbem_server_params), P(c_vp)])
_sig("fmmbem_submit", ctypes.c_int, [c_vp, P(fmmbem_mesh), P(c_d), ctypes.c_int, c_d, P(fmmbem_schedule),
                                     P(fmmbem_params), P(ctypes.c_uint64)])
_sig("fmmbem_poll", ctypes.c_int, [c_vp, ctypes.c_uint64, P(ctypes.c_int)])
_sig("fmmbem_wait", ctypes.c_int, [c_vp, ctypes.c_uint64, P(c_d), P(fmmbem_request_info)])
_sig("fmmbem_server_destroy", None, [c_vp])


class FmmbemError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"fmmbem error {code}: {what}")
        self.code = code


def fmmbem_last_error() -> str:
    return _lib.fmmbem_last_error().decode()


def _check(rc: int, allow=(OK,)) -> int:
    if rc not in allow:
        raise FmmbemError(rc, fmmbem_last_error())
    return rc


def _dp(a):
    return a.ctypes.data_as(P(c_d))


def _stream(stream):
    if stream is None:
        return c_vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return c_vp(stream.cuda_stream)
    return c_vp(int(stream))


def _dev_ptr(t: torch.Tensor, n: int, name: str):
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n):
        raise ValueError(f"{name} must be a contiguous CUDA float64 tensor with {n} elements")
    return c_vp(t.data_ptr())


def make_mesh(xyz, tri):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    m = fmmbem_mesh(xyz.shape[0], tri.shape[0], _dp(xyz), tri.ctypes.data_as(P(c_i32)))
    return m, (xyz, tri)


class DeviceAllocator:
    """Device memory for fmmbem_params.alloc/free from Python callables:
    alloc(nbytes) -> device address (int), free(address).  Keep the object
    alive as long as any context or request that uses it."""

    def __init__(self, alloc, free):
        self._alloc, self._free = alloc, free
        self.c_alloc = ALLOC_FN(lambda nbytes, _user: int(self._alloc(int(nbytes))) or None)
        self.c_free = FREE_FN(lambda ptr, _user: self._free(int(ptr)))


def torch_allocator(device=0) -> DeviceAllocator:
    """Device memory from PyTorch's caching allocator."""
    return DeviceAllocator(lambda n: torch.cuda.caching_allocator_alloc(n, device),
                           torch.cuda.caching_allocator_delete)


def params(theta=0.5, ncrit=64, p_max=16, mu=1.0, near_stored=0, m2l_stored=0, quad_far=4, quad_near=25,
           near_factor=2.0, allocator: DeviceAllocator | None = None) -> fmmbem_params:
    prm = fmmbem_params(theta, ncrit, p_max, mu, near_stored, m2l_stored, quad_far, quad_near, near_factor)
    if allocator is not None:
        prm.alloc, prm.free = allocator.c_alloc, allocator.c_free
        prm._allocator = allocator  # the callbacks live as long as the params
    return prm


def schedule(kernel=LAPLACE, **kw) -> fmmbem_schedule:
    s = fmmbem_schedule()
    _lib.fmmbem_schedule_default(ctypes.byref(s), kernel)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


class Context:
    """Owner of an fmmbem_ctx handle."""

    def __init__(self, handle, kernel, n):
        self.handle = handle
        self.kernel = kernel
        self.n = n

    def close(self):
        if self.handle:
            _lib.fmmbem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fmmbem_build(xyz, tri, kernel=LAPLACE, prm: fmmbem_params | None = None, stream=None) -> Context:
    m, keep = make_mesh(xyz, tri)
    h = c_vp()
    _check(_lib.fmmbem_build(ctypes.byref(m), kernel, ctypes.byref(prm) if prm is not None else None,
                             _stream(stream), ctypes.byref(h)))
    n = keep[1].shape[0] * (3 if kernel == STOKES else 1)
    return Context(h, kernel, n)


def fmmbem_matvec(ctx: Context, p: int, precision: int, x: torch.Tensor, y: torch.Tensor, stream=None):
    _check(_lib.fmmbem_matvec(ctx.handle, p, precision, _dev_ptr(x, ctx.n, "x"), _dev_ptr(y, ctx.n, "y"),
                              _stream(stream)))


def _report(cap: int):
    r = fmmbem_report()
    ph = np.zeros(cap, dtype=np.int32); pr = np.zeros(cap, dtype=np.uint8); rh = np.zeros(cap)
    r.hist_cap = cap
    r.p_hist = ph.ctypes.data_as(P(c_i32)); r.prec_hist = pr.ctypes.data_as(P(c_u8)); r.res_hist = _dp(rh)
    return r, (ph, pr, rh)


def _report_dict(r, bufs):
    ph, pr, rh = bufs
    k = min(r.iterations, r.hist_cap)
    return dict(iterations=r.iterations, restarts=r.restarts, converged=bool(r.converged), fallbacks=r.fallbacks,
                stalls=r.stalls, p_floor=r.p_floor,
                rel_res_implicit=r.rel_res_implicit, rel_res_true=r.rel_res_true, t_solve_s=r.t_solve_s,
                matvecs=r.matvecs, t_p2p_s=r.t_p2p_s, t_m2l_s=r.t_m2l_s, t_other_fmm_s=r.t_other_fmm_s,
                t_krylov_s=r.t_krylov_s, p_hist=ph[:k].copy(), prec_hist=pr[:k].copy(), res_hist=rh[:k].copy())


def fmmbem_solve_ctx(ctx: Context, b: torch.Tensor, tol: float, sched: fmmbem_schedule, x: torch.Tensor,
                     stream=None, hist_cap: int = 1000):
    r, bufs = _report(hist_cap)
    rc = _check(_lib.fmmbem_solve_ctx(ctx.handle, _dev_ptr(b, ctx.n, "b"), tol, ctypes.byref(sched),
                                      _dev_ptr(x, ctx.n, "x"), ctypes.byref(r), _stream(stream)),
                allow=(OK, ENOCONV))
    d = _report_dict(r, bufs)
    d["status"] = rc
    return d


def fmmbem_solve_ctx_static(ctx: Context, b: torch.Tensor, tol: float, sched: fmmbem_schedule, x: torch.Tensor,
                            stream=None, hist_cap: int = 1000):
    """fmmbem_solve_ctx with the Krylov workspace in the library's static
    device array: allocates nothing."""
    r, bufs = _report(hist_cap)
    rc = _check(_lib.fmmbem_solve_ctx_static(ctx.handle, _dev_ptr(b, ctx.n, "b"), tol, ctypes.byref(sched),
                                             _dev_ptr(x, ctx.n, "x"), ctypes.byref(r), _stream(stream)),
                allow=(OK, ENOCONV))
    d = _report_dict(r, bufs)
    d["status"] = rc
    return d


def fmmbem_solve(xyz, tri, bc, kernel, tol, sched: fmmbem_schedule, prm: fmmbem_params | None = None,
                 hist_cap: int = 1000):
    m, keep = make_mesh(xyz, tri)
    bc = np.ascontiguousarray(bc, dtype=np.float64)
    x = np.empty_like(bc)
    r, bufs = _report(hist_cap)
    rc = _check(_lib.fmmbem_solve(ctypes.byref(m), _dp(bc), kernel, tol, ctypes.byref(sched),
                                  ctypes.byref(prm) if prm is not None else None, _dp(x), ctypes.byref(r)),
                allow=(OK, ENOCONV))
    d = _report_dict(r, bufs)
    d["status"] = rc
    return x, d


def fmmbem_get_stats(ctx: Context) -> dict:
    s = fmmbem_stats()
    _check(_lib.fmmbem_get_stats(ctx.handle, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in fmmbem_stats._fields_}


def fmmbem_destroy(ctx: Context):
    ctx.close()


def fmmbem_set_timing(ctx: Context, enabled: bool):
    _check(_lib.fmmbem_set_timing(ctx.handle, int(bool(enabled))))


def fmmbem_set_timing_stages(ctx: Context, stages):
    """Time only the named stages (names of STAGES) or a bit mask."""
    mask = stages if isinstance(stages, int) else sum(1 << STAGES.index(s) for s in stages)
    _check(_lib.fmmbem_set_timing_stages(ctx.handle, mask))


def fmmbem_get_timing(ctx: Context, reset: bool = False):
    """{stage: (total ms, launches, algorithmic flops)} accumulated since the last reset."""
    t = np.zeros(N_STAGES); n = np.zeros(N_STAGES, dtype=np.int64); f = np.zeros(N_STAGES)
    _check(_lib.fmmbem_get_timing(ctx.handle, _dp(t), n.ctypes.data_as(P(c_i64)), _dp(f), int(bool(reset))))
    return {STAGES[i]: (float(t[i]), int(n[i]), float(f[i])) for i in range(N_STAGES)}


def fmmbem_tree(ctx: Context) -> dict:
    sz = np.zeros(4, dtype=np.int64)
    _check(_lib.fmmbem_tree_sizes(ctx.handle, sz.ctypes.data_as(P(c_i64))))
    nbox, nlev, nm, npp = (int(v) for v in sz)
    nt = ctx.n // (3 if ctx.kernel == STOKES else 1)
    out = dict(perm=np.empty(nt, np.int32), keys=np.empty(nt, np.uint64), boxes=np.empty((nbox, 6), np.int32),
               box_real=np.empty((nbox, 5)), m2l=np.empty((nm, 2), np.int32), p2p=np.empty((npp, 2), np.int32),
               cube=np.empty(4), nlevels=nlev)
    ip = lambda a: a.ctypes.data_as(P(c_i32))
    _check(_lib.fmmbem_tree_get(ctx.handle, ip(out["perm"]), out["keys"].ctypes.data_as(P(ctypes.c_uint64)),
                                ip(out["boxes"]), _dp(out["box_real"]), ip(out["m2l"]), ip(out["p2p"]),
                                _dp(out["cube"])))
    return out


class Server:
    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            _lib.fmmbem_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fmmbem_server_create(hbm_budget_bytes=8 << 30, max_active=16, n_streams=4) -> Server:
    p = fmmbem_server_params(hbm_budget_bytes, max_active, n_streams)
    h = c_vp()
    _check(_lib.fmmbem_server_create(ctypes.byref(p), ctypes.byref(h)))
    return Server(h)


def fmmbem_submit(srv: Server, xyz, tri, bc, kernel, tol, sched: fmmbem_schedule,
                  prm: fmmbem_params | None = None) -> int:
    m, keep = make_mesh(xyz, tri)
    bc = np.ascontiguousarray(bc, dtype=np.float64)
    t = ctypes.c_uint64()
    _check(_lib.fmmbem_submit(srv.handle, ctypes.byref(m), _dp(bc), kernel, tol, ctypes.byref(sched),
                              ctypes.byref(prm) if prm is not None else None, ctypes.byref(t)))
    return int(t.value)


def fmmbem_poll(srv: Server, ticket: int) -> bool:
    d = ctypes.c_int()
    _check(_lib.fmmbem_poll(srv.handle, ticket, ctypes.byref(d)))
    return bool(d.value)


def fmmbem_wait(srv: Server, ticket: int, n: int):
    x = np.empty(n)
    info = fmmbem_request_info()
    rc = _check(_lib.fmmbem_wait(srv.handle, ticket, _dp(x), ctypes.byref(info)), allow=(OK, ENOCONV))
    return x, {k: getattr(info, k) for k, _ in fmmbem_request_info._fields_} | {"status": rc}


def fmmbem_server_destroy(srv: Server):
    srv.close()
