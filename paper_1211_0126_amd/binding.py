"""Thin ctypes binding of libtmqcd.so (the C ABI in include/tmqcd.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch supplies device memory (the context's workspace, sized by
tm_workspace_bytes, and every input and output field) and the stream.
There is no CPU fallback: if the library is not built, loading it raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtmqcd.so")

TM_OK, TM_WARN_NOT_CONVERGED, TM_WARN_FALLBACK = 0, 1, 2
TM_EINVAL, TM_ENOMEM, TM_EDEVICE, TM_ESTATE, TM_ENOTSUP = -1, -2, -3, -4, -5
PREC_F64, PREC_F32, PREC_F16, PREC_BF16 = 0, 1, 2, 3
OP_M, OP_MDAG, OP_MDAGM, OP_HOP = 0, 1, 2, 3
LAYOUT_CANONICAL, LAYOUT_NATIVE = 0, 1
STOP_NORMAL, STOP_TRUE = 0, 1
SOLVER_CG, SOLVER_FCG_LEARNED, SOLVER_CG_EO = 0, 1, 2
LOOP_STANDARD, LOOP_ONEEND_ISOVECTOR, LOOP_ONEEND_GENERALIZED, LOOP_DERIVATIVE = 0, 1, 2, 3
ALL_MOMENTA = -1
KC_NAMES = ["dslash", "dslash_upd", "blas", "contract", "other", "apply", "eo_hop", "eo_hop_dag"]


class TmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("tmqcd error %d: %s" % (code, msg))
        self.code = code


class Lattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("kappa", ctypes.c_double), ("mu", ctypes.c_double),
                ("t_bc", ctypes.c_int32)]


class SolveParams(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("solver", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("stop", ctypes.c_int32), ("reliable", ctypes.c_int32),
                ("delta", ctypes.c_double), ("rhs_block", ctypes.c_int32), ("true_resid", ctypes.c_int32),
                ("out_layout", ctypes.c_int32), ("out_prec", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("truncated", ctypes.c_int32),
                ("fell_back", ctypes.c_int32), ("resid_iterated", ctypes.c_double), ("resid_true", ctypes.c_double)]


class TsmParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_hp", ctypes.c_int32), ("n_lp", ctypes.c_int32),
                ("lp", SolveParams), ("hp", SolveParams), ("n_mom", ctypes.c_int32),
                ("mom_host", ctypes.POINTER(ctypes.c_int32)), ("estimator", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


CAPS_MAX_SOLVES = 4


class Caps(ctypes.Structure):
    _fields_ = [("n_solves", ctypes.c_int32), ("solves", SolveParams * CAPS_MAX_SOLVES),
                ("max_sources", ctypes.c_int32), ("max_mom", ctypes.c_int32), ("mom_distinct", ctypes.c_int32),
                ("estimators", ctypes.c_uint32), ("all_mom_sources", ctypes.c_int32), ("field_rhs", ctypes.c_int32),
                ("train_pairs", ctypes.c_int32), ("train_sources", ctypes.c_int32), ("loss_pairs", ctypes.c_int32)]


def caps(solves=(), max_sources=64, max_mom=27, mom_distinct=3, estimators=(LOOP_STANDARD,), all_mom_sources=0,
         field_rhs=1, train_pairs=0, train_sources=0, loss_pairs=0) -> Caps:
    """What a context will be asked to do (tm_caps): the solve settings (at
    most four SolveParams), and the per-call maxima of the other calls."""
    solves = list(solves)
    assert len(solves) <= CAPS_MAX_SOLVES
    c = Caps()
    c.n_solves = len(solves)
    for i, sp in enumerate(solves):
        c.solves[i] = sp
    c.max_sources, c.max_mom, c.mom_distinct = int(max_sources), int(max_mom), int(mom_distinct)
    c.estimators = sum(1 << int(e) for e in estimators)
    c.all_mom_sources, c.field_rhs = int(all_mom_sources), int(field_rhs)
    c.train_pairs, c.train_sources, c.loss_pairs = int(train_pairs), int(train_sources), int(loss_pairs)
    return c


class RunStats(ctypes.Structure):
    _fields_ = [("ms_hp_phase", ctypes.c_double), ("ms_lp_phase", ctypes.c_double), ("lp_iters", ctypes.c_int64),
                ("hp_iters", ctypes.c_int64), ("max_lp_resid_true", ctypes.c_double),
                ("max_hp_resid_true", ctypes.c_double), ("hp_not_converged", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


EXPORTS = [
    "tm_abi_version", "tm_create", "tm_destroy", "tm_last_error", "tm_gauge_load", "tm_field_bytes",
    "tm_field_convert", "tm_dslash", "tm_dslash_noalloc", "tm_noise_z4", "tsm_solve_batch", "tsm_contract", "tsm_contract_est",
    "tsm_loops",
    "tm_profile_enable", "tm_profile_read", "tm_workspace_bytes", "tm_workspace_usage",
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtmqcd.so; raises if it is not built (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libtmqcd.so is not built (%s); run __graft_entry__.build()" % path)
    # torch ships its own HIP/HSA runtime libraries; load them first so that
    # the library binds to the same runtime (two runtimes in one process do
    # not see the device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, i32, u64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.tm_abi_version.restype = i32
    lib.tm_create.argtypes = [ctypes.POINTER(Lattice), P, ctypes.c_size_t, P, ctypes.POINTER(P)]
    lib.tm_workspace_bytes.argtypes = [ctypes.POINTER(Lattice), ctypes.POINTER(Caps)]
    lib.tm_workspace_bytes.restype = ctypes.c_size_t
    lib.tm_workspace_usage.argtypes = [P, P, P, P]
    lib.tm_destroy.argtypes = [P]
    lib.tm_last_error.argtypes = [P]
    lib.tm_last_error.restype = ctypes.c_char_p
    lib.tm_gauge_load.argtypes = [P, P]
    lib.tm_field_bytes.argtypes = [P, i32, i32, i32]
    lib.tm_field_bytes.restype = ctypes.c_size_t
    lib.tm_field_convert.argtypes = [P, i32, i32, i32, P, P]
    lib.tm_dslash.argtypes = [P, i32, i32, i32, i32, P, P]
    lib.tm_dslash_noalloc.argtypes = [P, i32, i32, i32, i32, P, P]
    lib.tm_noise_z4.argtypes = [P, u64, i32, P, P]
    lib.tsm_solve_batch.argtypes = [P, ctypes.POINTER(SolveParams), u64, i32, P, P, P]
    lib.tsm_contract.argtypes = [P, u64, i32, P, P, i32, P, P]
    lib.tsm_contract_est.argtypes = [P, i32, u64, i32, P, P, i32, P, P]
    lib.tsm_loops.argtypes = [P, ctypes.POINTER(TsmParams), P, P, P, P, ctypes.POINTER(RunStats)]
    lib.tm_profile_enable.argtypes = [P, i32]
    lib.tm_profile_read.argtypes = [P, P, P, P]
    for name in EXPORTS:
        if name not in ("tm_abi_version", "tm_last_error", "tm_field_bytes", "tm_workspace_bytes"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def solve_params(prec=PREC_F64, tol=1e-10, max_iter=-1, stop=STOP_NORMAL, reliable=0, delta=0.1, rhs_block=0,
                 true_resid=1, solver=SOLVER_CG, out_layout=LAYOUT_CANONICAL, out_prec=PREC_F64) -> SolveParams:
    return SolveParams(prec, solver, tol, max_iter, stop, reliable, delta, rhs_block, true_resid, out_layout,
                       out_prec)


def _lattice(dims, kappa, mu, t_bc) -> Lattice:
    return Lattice((ctypes.c_int32 * 4)(*[int(d) for d in dims]), float(kappa), float(mu), int(t_bc))


def tm_workspace_bytes(dims, kappa=0.1, mu=0.0, t_bc=-1, caps_=None) -> int:
    """Workspace bytes for a context of this lattice doing what caps_ (a
    Caps; None: every solver and precision at 32 sources per block)
    describes; 0 for a lattice tm_create refuses."""
    lat = _lattice(dims, kappa, mu, t_bc)
    return int(load_library().tm_workspace_bytes(ctypes.byref(lat), ctypes.byref(caps_) if caps_ is not None
                                                 else None))


class Context:
    """One lattice on the current device; wraps a tm_ctx* and owns its
    workspace (a torch uint8 tensor of tm_workspace_bytes(caps) bytes, or of
    workspace_bytes if given)."""

    def __init__(self, dims, kappa, mu, t_bc=-1, stream=None, caps=None, workspace_bytes=None):
        import torch
        self.lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.kappa, self.mu, self.t_bc = float(kappa), float(mu), int(t_bc)
        self.V = int(np.prod(self.dims))
        lat = _lattice(self.dims, kappa, mu, t_bc)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        if workspace_bytes is None:
            workspace_bytes = int(self.lib.tm_workspace_bytes(ctypes.byref(lat),
                                                              ctypes.byref(caps) if caps is not None else None))
            if workspace_bytes == 0:
                self.lib.tm_create(ctypes.byref(lat), None, 0, None, ctypes.byref(ctypes.c_void_p()))
                raise TmError(TM_EINVAL, self.lib.tm_last_error(None).decode())
        self.workspace = torch.empty(max(int(workspace_bytes), 1), dtype=torch.uint8, device="cuda")
        h = ctypes.c_void_p()
        rc = self.lib.tm_create(ctypes.byref(lat), ctypes.c_void_p(self.workspace.data_ptr()),
                                int(workspace_bytes), ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if rc != TM_OK:
            self.workspace = None
            raise TmError(rc, self.lib.tm_last_error(None).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.tm_destroy(self.h)  # waits for the context's stream
            self.h = None
        self.workspace = None

    def workspace_usage(self) -> dict:
        """Bytes held until close (persistent), the most scratch one call has
        used (peak_scratch), and the workspace size (total)."""
        v = [ctypes.c_size_t() for _ in range(3)]
        self.check(self.lib.tm_workspace_usage(self.h, *[ctypes.byref(x) for x in v]))
        return {"persistent": v[0].value, "peak_scratch": v[1].value, "total": v[2].value}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc, allow_warn=True):
        if rc < 0 or (rc > 0 and not allow_warn):
            raise TmError(rc, self.lib.tm_last_error(self.h).decode())
        return rc


def tm_abi_version() -> int:
    return int(load_library().tm_abi_version())


def tm_create(dims, kappa, mu, t_bc=-1, stream=None, caps=None, workspace_bytes=None) -> Context:
    return Context(dims, kappa, mu, t_bc, stream, caps, workspace_bytes)


def tm_gauge_load(ctx: Context, links: np.ndarray) -> None:
    links = np.ascontiguousarray(links, dtype=np.complex128)
    assert links.shape == (ctx.V, 4, 3, 3)
    ctx.check(ctx.lib.tm_gauge_load(ctx.h, _ptr(links)))


def _canon_dtype(prec):
    import torch
    return {PREC_F64: torch.complex128, PREC_F32: torch.complex64, PREC_F16: torch.float16,
            PREC_BF16: torch.bfloat16}[prec]


def canonical_shape(ctx: Context, prec, nrhs):
    if prec in (PREC_F16, PREC_BF16):
        return (nrhs, ctx.V, 4, 3, 2)
    return (nrhs, ctx.V, 4, 3)


def tm_field_bytes(ctx: Context, prec, nrhs, layout) -> int:
    return int(ctx.lib.tm_field_bytes(ctx.h, prec, nrhs, layout))


def tm_field_convert(ctx: Context, prec, nrhs, to_native, x, out):
    ctx.check(ctx.lib.tm_field_convert(ctx.h, prec, nrhs, int(to_native), ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr())))
    return out


def tm_dslash(ctx: Context, op, prec, x, out=None, layout=LAYOUT_CANONICAL, nrhs=None):
    """out = op(x) for canonical tensors [nrhs][V][4][3] (complex) or
    [nrhs][V][4][3][2] (F16/BF16 pairs), or native uint8 buffers."""
    import torch
    if layout == LAYOUT_CANONICAL:
        nrhs = x.shape[0]
        assert tuple(x.shape) == canonical_shape(ctx, prec, nrhs) and x.dtype == _canon_dtype(prec)
        assert x.is_cuda and x.is_contiguous()
        if out is None:
            out = torch.empty_like(x)
    else:
        assert nrhs is not None and out is not None
    ctx.check(ctx.lib.tm_dslash(ctx.h, op, prec, nrhs, layout, ctypes.c_void_p(x.data_ptr()),
                                ctypes.c_void_p(out.data_ptr())))
    return out


def tm_dslash_noalloc(ctx: Context, op, prec, x, out, layout=LAYOUT_CANONICAL, nrhs=None):
    """out = op(x) through the allocation-free entry point; out is the
    caller's tensor (nothing is allocated here either)."""
    if layout == LAYOUT_CANONICAL:
        nrhs = x.shape[0]
        assert tuple(x.shape) == canonical_shape(ctx, prec, nrhs) and x.dtype == _canon_dtype(prec)
        assert tuple(out.shape) == tuple(x.shape) and out.dtype == x.dtype
        assert x.is_cuda and x.is_contiguous() and out.is_cuda and out.is_contiguous()
    else:
        assert nrhs is not None
    ctx.check(ctx.lib.tm_dslash_noalloc(ctx.h, op, prec, nrhs, layout, ctypes.c_void_p(x.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr())))
    return out


def tm_noise_z4(ctx: Context, seed, ids):
    import torch
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
    out = torch.empty((len(ids), ctx.V, 4, 3), dtype=torch.complex128, device="cuda")
    ctx.check(ctx.lib.tm_noise_z4(ctx.h, int(seed), len(ids), _ptr(ids), ctypes.c_void_p(out.data_ptr())))
    return out


def _stats_list(st):
    return [{"iters": s.iters, "converged": bool(s.converged), "truncated": bool(s.truncated),
             "fell_back": bool(s.fell_back), "resid_iterated": s.resid_iterated, "resid_true": s.resid_true}
            for s in st]


def tsm_solve_batch(ctx: Context, params: SolveParams, seed, ids, want_solutions=True):
    """Returns (solutions on the device or None, stats list, status).  The
    solutions follow params.out_layout / out_prec: canonical [n][V][4][3]
    complex128 / complex64 (or [n][V][4][3][2] binary16 / bfloat16 pairs),
    or a native uint8 buffer of tm_field_bytes(ctx, out_prec, n, NATIVE)."""
    import torch
    ids = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64))
    n = len(ids)
    sol = None
    if want_solutions:
        if params.out_layout == LAYOUT_NATIVE:
            sol = torch.empty(max(tm_field_bytes(ctx, params.out_prec, n, LAYOUT_NATIVE), 1), dtype=torch.uint8,
                              device="cuda")
        else:
            sol = torch.empty(canonical_shape(ctx, params.out_prec, n), dtype=_canon_dtype(params.out_prec),
                              device="cuda")
    st = (SolveStats * max(n, 1))()
    rc = ctx.lib.tsm_solve_batch(ctx.h, ctypes.byref(params), int(seed), n, _ptr(ids),
                                 ctypes.c_void_p(sol.data_ptr()) if sol is not None else None, st)
    ctx.check(rc)
    return sol, _stats_list(st[:n]), rc


def tsm_contract(ctx: Context, seed, ids, sol, mom, estimator=LOOP_STANDARD):
    """Loops of given solutions, complex128 [n][16][n_mom][Lt] (host).  The
    one-end estimators ignore seed and ids (pass ids=None and the count comes
    from sol).  mom=None projects the standard loop onto every momentum of
    the lattice: [n][16][Lx*Ly*Lz][Lt]."""
    import torch
    n = len(ids) if ids is not None else int(sol.shape[0])
    ids_a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint64)) if ids is not None else None
    if mom is None:
        # every momentum of the lattice, index nx + Lx (ny + Ly nz)
        n_mom, mom_p = ALL_MOMENTA, None
        el = (16, ctx.dims[0] * ctx.dims[1] * ctx.dims[2], ctx.dims[3])
    else:
        mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
        n_mom, mom_p = mom.shape[0], _ptr(mom)
        el = (4, 16, n_mom, ctx.dims[3]) if estimator == LOOP_DERIVATIVE else (16, n_mom, ctx.dims[3])
    out = np.zeros((n,) + el, dtype=np.complex128)
    assert sol.is_cuda and sol.is_contiguous() and tuple(sol.shape) == (n, ctx.V, 4, 3)
    assert sol.dtype == torch.complex128
    ctx.check(ctx.lib.tsm_contract_est(ctx.h, int(estimator), int(seed), n,
                                       _ptr(ids_a) if ids_a is not None else None,
                                       ctypes.c_void_p(sol.data_ptr()), n_mom, mom_p, _ptr(out)))
    return out


def tsm_loops(ctx: Context, seed, n_hp, n_lp, lp: SolveParams, hp: SolveParams, mom, per_source=False,
              stats=True, estimator=LOOP_STANDARD):
    """The TSM estimate (Eq. 4).  Returns dict with 'loops' [3][16][n_mom][Lt]
    (C, B, T), 'err', optional 'per_source' [N][2][16][n_mom][Lt], 'stats'
    (list of [LP, HP] records), 'run' and the status code; the derivative
    estimator has [4][16][n_mom][Lt] in place of each [16][n_mom][Lt]."""
    mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    nm, lt = mom.shape[0], ctx.dims[3]
    N = n_hp + n_lp
    P = TsmParams(int(seed), int(n_hp), int(n_lp), lp, hp, nm, mom.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                  int(estimator), 0)
    el = (4, 16, nm, lt) if estimator == LOOP_DERIVATIVE else (16, nm, lt)
    loops = np.zeros((3,) + el, dtype=np.complex128)
    err = np.zeros_like(loops)
    ps = np.zeros((max(N, 1), 2) + el, dtype=np.complex128) if per_source else None
    st = (SolveStats * (2 * max(N, 1)))() if stats else None
    run = RunStats()
    rc = ctx.lib.tsm_loops(ctx.h, ctypes.byref(P), _ptr(loops), _ptr(err), _ptr(ps) if ps is not None else None,
                           st, ctypes.byref(run))
    ctx.check(rc)
    res = {"loops": loops, "err": err, "status": rc,
           "run": {f: getattr(run, f) for f, _ in RunStats._fields_}}
    if ps is not None:
        res["per_source"] = ps[:N]
    if st is not None:
        sl = _stats_list(st[:2 * N])
        res["stats"] = [[sl[2 * j], sl[2 * j + 1]] for j in range(N)]
    return res


def tm_profile_enable(ctx: Context, on=True):
    ctx.check(ctx.lib.tm_profile_enable(ctx.h, 1 if on else 0))


def tm_profile_read(ctx: Context):
    n = len(KC_NAMES)
    la = np.zeros(n, dtype=np.int64)
    ms = np.zeros(n, dtype=np.float64)
    by = np.zeros(n, dtype=np.float64)
    ctx.check(ctx.lib.tm_profile_read(ctx.h, _ptr(la), _ptr(ms), _ptr(by)))
    return {KC_NAMES[k]: {"launches": int(la[k]), "ms": float(ms[k]), "bytes": float(by[k])} for k in range(n)}


# ---- learned preconditioner ------------------------------------------------

NET_MAX_LAYERS = 8


class NetShape(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int32), ("widths", ctypes.c_int32 * (NET_MAX_LAYERS + 1))]


class TrainParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("n_sources", ctypes.c_int32), ("n_pairs", ctypes.c_int32),
                ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("hp_tol", ctypes.c_double), ("min_rel_err", ctypes.c_double), ("init_seed", ctypes.c_uint64),
                ("init_scale", ctypes.c_double), ("init_mode", ctypes.c_int32), ("loss_mode", ctypes.c_int32)]


class TrainStats(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double), ("ms_generate", ctypes.c_double),
                ("ms_train", ctypes.c_double), ("pairs", ctypes.c_int32), ("steps", ctypes.c_int32)]


def _net_shape(widths) -> NetShape:
    w = list(widths) + [0] * (NET_MAX_LAYERS + 1 - len(widths))
    return NetShape(len(widths) - 1, (ctypes.c_int32 * (NET_MAX_LAYERS + 1))(*w))


def _learn_sigs(lib):
    P, i32 = ctypes.c_void_p, ctypes.c_int32
    lib.tm_precond_weight_count.argtypes = [ctypes.POINTER(NetShape)]
    lib.tm_precond_weight_count.restype = ctypes.c_size_t
    lib.tm_precond_set.argtypes = [P, ctypes.POINTER(NetShape), P]
    lib.tm_precond_set.restype = i32
    lib.tm_precond_get.argtypes = [P, ctypes.POINTER(NetShape), P]
    lib.tm_precond_get.restype = i32
    lib.tm_precond_apply.argtypes = [P, i32, i32, P, P]
    lib.tm_precond_apply.restype = i32
    lib.tm_precond_loss_grad.argtypes = [P, i32, P, P, P, P]
    lib.tm_precond_loss_grad.restype = i32
    lib.tm_precond_train.argtypes = [P, ctypes.POINTER(TrainParams), ctypes.POINTER(TrainStats)]
    lib.tm_precond_train.restype = i32


EXPORTS += ["tm_precond_weight_count", "tm_precond_set", "tm_precond_get", "tm_precond_apply",
            "tm_precond_loss_grad", "tm_precond_train"]


def tm_precond_weight_count(widths) -> int:
    lib = load_library()
    _learn_sigs(lib)
    return int(lib.tm_precond_weight_count(ctypes.byref(_net_shape(widths))))


def tm_precond_set(ctx: Context, widths, weights: np.ndarray) -> None:
    _learn_sigs(ctx.lib)
    w = np.ascontiguousarray(weights, dtype=np.complex128)
    assert w.size == tm_precond_weight_count(widths)
    ctx.check(ctx.lib.tm_precond_set(ctx.h, ctypes.byref(_net_shape(widths)), _ptr(w)))


def tm_precond_get(ctx: Context):
    _learn_sigs(ctx.lib)
    sh = NetShape()
    ctx.check(ctx.lib.tm_precond_get(ctx.h, ctypes.byref(sh), None))
    widths = [sh.widths[i] for i in range(sh.n_layers + 1)]
    w = np.zeros(tm_precond_weight_count(widths), dtype=np.complex128)
    ctx.check(ctx.lib.tm_precond_get(ctx.h, ctypes.byref(sh), _ptr(w)))
    return widths, w


def tm_precond_apply(ctx: Context, x, adjoint=False):
    """N(x) or N^dag(x) for canonical complex128 [n][V][4][3] device tensors."""
    import torch
    _learn_sigs(ctx.lib)
    assert x.dtype == torch.complex128 and x.is_cuda and x.is_contiguous()
    out = torch.empty_like(x)
    ctx.check(ctx.lib.tm_precond_apply(ctx.h, 1 if adjoint else 0, x.shape[0], ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr())))
    return out


def tm_precond_loss_grad(ctx: Context, r, e):
    """Loss and Wirtinger gradient (d/d conj W) of pairs given as device tensors."""
    _learn_sigs(ctx.lib)
    widths, w = tm_precond_get(ctx)
    loss = ctypes.c_double()
    grad = np.zeros_like(w)
    ctx.check(ctx.lib.tm_precond_loss_grad(ctx.h, r.shape[0], ctypes.c_void_p(r.data_ptr()),
                                           ctypes.c_void_p(e.data_ptr()), ctypes.byref(loss), _ptr(grad)))
    return loss.value, grad


def tm_precond_train(ctx: Context, seed, n_sources, n_pairs, epochs, batch, lr=1e-3, hp_tol=1e-10,
                     min_rel_err=1e-4, init_seed=1, init_scale=1e-2, init_mode=1, loss_mode=1):
    """init_mode 0: identity start; 1: third-order Neumann series of M^{-1}.
    loss_mode 0: error loss; 1: residual loss.  n_pairs = epochs = 0
    installs the initial network only."""
    _learn_sigs(ctx.lib)
    p = TrainParams(int(seed), int(n_sources), int(n_pairs), int(epochs), int(batch), float(lr), float(hp_tol),
                    float(min_rel_err), int(init_seed), float(init_scale), int(init_mode), int(loss_mode))
    st = TrainStats()
    ctx.check(ctx.lib.tm_precond_train(ctx.h, ctypes.byref(p), ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in TrainStats._fields_}


# ---- tuning ------------------------------------------------------------------

EXPORTS += ["tm_autotune", "tm_set_lane_rhs"]


def tm_autotune(ctx: Context, prec, nrhs):
    """Returns (best right-hand sides per lane, ms per application for 1, 2, 4)."""
    ctx.lib.tm_autotune.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p]
    ctx.lib.tm_autotune.restype = ctypes.c_int32
    best = ctypes.c_int32()
    ms = np.zeros(3, dtype=np.float64)
    ctx.check(ctx.lib.tm_autotune(ctx.h, int(prec), int(nrhs), ctypes.byref(best), _ptr(ms)))
    return int(best.value), ms


def tm_set_lane_rhs(ctx: Context, prec, nr):
    ctx.lib.tm_set_lane_rhs.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
    ctx.lib.tm_set_lane_rhs.restype = ctypes.c_int32
    ctx.check(ctx.lib.tm_set_lane_rhs(ctx.h, int(prec), int(nr)))
