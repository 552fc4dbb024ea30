"""ctypes wrapper around the plain C oracle (tm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU
baseline of the benchmark.  Arrays are numpy complex128 in the canonical
layouts: gauge [V][4][3][3], spinor [V][4][3].
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tm_oracle.c")
_LIB = os.path.join(_HERE, "libtmoracle.so")

OP_M, OP_MDAG, OP_MDAGM, OP_HOP = 0, 1, 2, 3
STOP_NORMAL, STOP_TRUE = 0, 1
LOOP_STD, LOOP_ONEEND_VV, LOOP_ONEEND_GEN, LOOP_DERIV = 0, 1, 2, 3

_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile tm_oracle.c with gcc into oracle/libtmoracle.so."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def load_oracle():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_oracle()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, f64, u64 = ctypes.c_int, ctypes.c_double, ctypes.c_uint64
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_get_threads.restype = i32
    lib.orc_gamma.argtypes = [i32, P]
    lib.orc_gamma_mu.argtypes = [i32, P]
    lib.orc_splitmix64_next.argtypes = [ctypes.POINTER(u64)]
    lib.orc_splitmix64_next.restype = u64
    lib.orc_noise_hash.argtypes = [u64, u64, u64, u64]
    lib.orc_noise_hash.restype = u64
    lib.orc_noise_codes.argtypes = [P, u64, u64, P]
    lib.orc_noise_z4.argtypes = [P, u64, u64, P]
    lib.orc_apply.argtypes = [P, i32, f64, f64, i32, P, P, P]
    lib.orc_cgnr.argtypes = [P, i32, f64, f64, P, P, f64, i32, i32, P, P]
    lib.orc_cgnr.restype = i32
    lib.orc_loops.argtypes = [P, P, P, i32, P, P]
    lib.orc_loops_deriv.argtypes = [P, i32, P, P, P, i32, P, P]
    lib.orc_loops_est.argtypes = [P, i32, f64, f64, P, i32, P, P, i32, P, P]
    lib.orc_tsm.argtypes = [P, i32, f64, f64, P, u64, i32, i32, f64, i32, i32, f64, i32, i32,
                            i32, P, i32, P, P, P, P, i32, i32]
    lib.orc_eo_apply.argtypes = [P, i32, f64, f64, i32, P, P, P]
    lib.orc_eo_apply.restype = i32
    lib.orc_eo_source.argtypes = [P, i32, f64, f64, P, P, P]
    lib.orc_eo_reconstruct.argtypes = [P, i32, f64, f64, P, P, P]
    lib.orc_cgnr_eo.argtypes = [P, i32, f64, f64, P, P, f64, i32, i32, P, P]
    lib.orc_cgnr_eo.restype = i32
    lib.orc_tsm.restype = i32
    lib.orc_pt_layer.argtypes = [P, i32, P, i32, i32, P, P, P]
    lib.orc_pt_layer_adj.argtypes = [P, i32, P, i32, i32, P, P, P]
    lib.orc_pt_net.argtypes = [P, i32, P, i32, P, P, P, P, i32]
    lib.orc_pt_loss_grad.argtypes = [P, i32, P, i32, P, P, i32, P, P, P]
    lib.orc_pt_loss_grad.restype = f64
    lib.orc_fcg.argtypes = [P, i32, f64, f64, P, i32, P, P, P, f64, i32, P, P]
    lib.orc_fcg.restype = i32
    lib.orc_fgmres.argtypes = [P, i32, f64, f64, P, i32, P, P, P, f64, i32, i32, P, P]
    lib.orc_fgmres.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def set_threads(n: int) -> None:
    load_oracle().orc_set_threads(int(n))


def get_threads() -> int:
    return int(load_oracle().orc_get_threads())


def gamma(n: int) -> np.ndarray:
    out = np.zeros((4, 4), dtype=np.complex128)
    load_oracle().orc_gamma(int(n), _ptr(out))
    return out


def gamma_mu(mu: int) -> np.ndarray:
    """gamma_mu for mu = 0..3 (x, y, z, t) and gamma_5 for mu = 4."""
    out = np.zeros((4, 4), dtype=np.complex128)
    load_oracle().orc_gamma_mu(int(mu), _ptr(out))
    return out


def splitmix64_sequence(state: int, n: int) -> list:
    st = ctypes.c_uint64(state)
    lib = load_oracle()
    return [int(lib.orc_splitmix64_next(ctypes.byref(st))) for _ in range(n)]


def noise_hash(seed: int, j: int, vol: int, site: int) -> int:
    return int(load_oracle().orc_noise_hash(seed, j, vol, site))


def noise_codes(dims, seed: int, j: int) -> np.ndarray:
    d = _dims(dims)
    v = int(np.prod(d))
    out = np.zeros((v, 12), dtype=np.uint8)
    load_oracle().orc_noise_codes(_ptr(d), seed, j, _ptr(out))
    return out


def noise_z4(dims, seed: int, j: int) -> np.ndarray:
    d = _dims(dims)
    v = int(np.prod(d))
    out = np.zeros((v, 4, 3), dtype=np.complex128)
    load_oracle().orc_noise_z4(_ptr(d), seed, j, _ptr(out))
    return out


def apply_op(dims, t_bc, kappa, mu, op, U, psi) -> np.ndarray:
    d = _dims(dims)
    U = _c128(U)
    psi = _c128(psi)
    out = np.zeros_like(psi)
    load_oracle().orc_apply(_ptr(d), int(t_bc), float(kappa), float(mu), int(op), _ptr(U), _ptr(psi), _ptr(out))
    return out


def cgnr(dims, t_bc, kappa, mu, U, eta, tol, maxit=-1, stop=STOP_NORMAL):
    """Returns (solution, stats dict)."""
    d = _dims(dims)
    U = _c128(U)
    eta = _c128(eta)
    x = np.zeros_like(eta)
    st = np.zeros(5, dtype=np.float64)
    load_oracle().orc_cgnr(_ptr(d), int(t_bc), float(kappa), float(mu), _ptr(U), _ptr(eta), float(tol),
                           int(maxit), int(stop), _ptr(x), _ptr(st))
    return x, {"iters": int(st[0]), "resid_normal": st[1], "resid_true": st[2],
               "converged": bool(st[3]), "truncated": bool(st[4])}


def eo_apply(dims, t_bc, kappa, mu, op, U, psi) -> np.ndarray:
    """The even-odd Schur complement Mhat = M_oo - M_oe M_ee^{-1} M_eo (op 0),
    its adjoint (op 1) or Mhat^dag Mhat (op 2) on a full-size field whose odd
    sites are used; the result is zero on the even sites.  Every extent must
    be even."""
    d = _dims(dims)
    psi = _c128(psi)
    out = np.zeros_like(psi)
    rc = load_oracle().orc_eo_apply(_ptr(d), int(t_bc), float(kappa), float(mu), int(op), _ptr(_c128(U)),
                                    _ptr(psi), _ptr(out))
    if rc != 0:
        raise ValueError("even-odd reduction needs even extents")
    return out


def eo_source(dims, t_bc, kappa, mu, U, eta) -> np.ndarray:
    """etahat_o = eta_o - M_oe M_ee^{-1} eta_e (zero on the even sites)."""
    d = _dims(dims)
    eta = _c128(eta)
    out = np.zeros_like(eta)
    load_oracle().orc_eo_source(_ptr(d), int(t_bc), float(kappa), float(mu), _ptr(_c128(U)), _ptr(eta), _ptr(out))
    return out


def eo_reconstruct(dims, t_bc, kappa, mu, U, eta, x_odd) -> np.ndarray:
    """The whole solution from its odd half: x_e = M_ee^{-1}(eta_e - M_eo x_o)."""
    d = _dims(dims)
    x = np.array(_c128(x_odd), copy=True)
    load_oracle().orc_eo_reconstruct(_ptr(d), int(t_bc), float(kappa), float(mu), _ptr(_c128(U)),
                                     _ptr(_c128(eta)), _ptr(x))
    return x


def cgnr_eo(dims, t_bc, kappa, mu, U, eta, tol, maxit=-1, stop=STOP_NORMAL):
    """CG on the normal equations of the even-odd Schur complement, then the
    even half reconstructed.  Returns (solution, stats dict); resid_normal is
    that of the Schur normal equations."""
    d = _dims(dims)
    U = _c128(U)
    eta = _c128(eta)
    x = np.zeros_like(eta)
    st = np.zeros(5, dtype=np.float64)
    rc = load_oracle().orc_cgnr_eo(_ptr(d), int(t_bc), float(kappa), float(mu), _ptr(U), _ptr(eta), float(tol),
                                   int(maxit), int(stop), _ptr(x), _ptr(st))
    if rc < 0:
        raise ValueError("even-odd reduction needs even extents")
    return x, {"iters": int(st[0]), "resid_normal": st[1], "resid_true": st[2],
               "converged": bool(st[3]), "truncated": bool(st[4])}


def loops(dims, eta, s, mom) -> np.ndarray:
    """complex128 [16][n_mom][Lt]."""
    d = _dims(dims)
    mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((16, mom.shape[0], int(d[3])), dtype=np.complex128)
    load_oracle().orc_loops(_ptr(d), _ptr(_c128(eta)), _ptr(_c128(s)), mom.shape[0], _ptr(mom), _ptr(out))
    return out


def loops_deriv(dims, t_bc, U, eta, s, mom) -> np.ndarray:
    """One-derivative loops (symmetric covariant derivative in each
    direction mu): complex128 [4][16][n_mom][Lt]."""
    d = _dims(dims)
    mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((4, 16, mom.shape[0], int(d[3])), dtype=np.complex128)
    load_oracle().orc_loops_deriv(_ptr(d), int(t_bc), _ptr(_c128(U)), _ptr(_c128(eta)), _ptr(_c128(s)),
                                  mom.shape[0], _ptr(mom), _ptr(out))
    return out


def loops_est(dims, t_bc, kappa, mu, U, est, s, mom, eta=None) -> np.ndarray:
    """Loops of estimator est (LOOP_STD needs eta; the one-end estimators of
    section 2.3, Eqs. 5 and 6, use the solution alone): complex128
    [16][n_mom][Lt]."""
    d = _dims(dims)
    mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    out = np.zeros((16, mom.shape[0], int(d[3])), dtype=np.complex128)
    if est == LOOP_DERIV:
        return loops_deriv(dims, t_bc, U, eta, s, mom)
    if est == LOOP_STD and eta is None:
        raise ValueError("the standard loop needs the source")
    e = _c128(eta) if eta is not None else None
    load_oracle().orc_loops_est(_ptr(d), int(t_bc), float(kappa), float(mu), _ptr(_c128(U)), int(est),
                                _ptr(e) if e is not None else None, _ptr(_c128(s)), mom.shape[0], _ptr(mom),
                                _ptr(out))
    return out


def tsm(dims, t_bc, kappa, mu, U, seed, n_hp, n_lp, lp_tol, lp_maxit, hp_tol, hp_maxit, mom,
        lp_stop=STOP_NORMAL, hp_stop=STOP_NORMAL, per_source=False, estimator=LOOP_STD, lp_eo=False, hp_eo=False):
    """Returns dict with 'loops' [3][16][n_mom][Lt] (C, B, T), 'err', optional
    'per_source' [N][2][16][n_mom][Lt] and 'stats' [N][2][5].  lp_eo / hp_eo
    solve that set on the even-odd Schur complement."""
    d = _dims(dims)
    U = _c128(U)
    mom = np.ascontiguousarray(np.asarray(mom, dtype=np.int32).reshape(-1, 3))
    nm = mom.shape[0]
    lt = int(d[3])
    el = (4, 16, nm, lt) if estimator == LOOP_DERIV else (16, nm, lt)
    out = np.zeros((3,) + el, dtype=np.complex128)
    err = np.zeros_like(out)
    n = n_hp + n_lp
    ps = np.zeros((max(n, 1), 2) + el, dtype=np.complex128) if per_source else None
    st = np.zeros((max(n, 1), 2, 5), dtype=np.float64)
    load_oracle().orc_tsm(_ptr(d), int(t_bc), float(kappa), float(mu), _ptr(U), int(seed), int(n_hp), int(n_lp),
                          float(lp_tol), int(lp_maxit), int(lp_stop), float(hp_tol), int(hp_maxit), int(hp_stop),
                          nm, _ptr(mom), int(estimator), _ptr(out), _ptr(err), _ptr(ps) if ps is not None else None,
                          _ptr(st), int(bool(lp_eo)), int(bool(hp_eo)))
    res = {"loops": out, "err": err, "stats": st[:n]}
    if ps is not None:
        res["per_source"] = ps[:n]
    return res


# ---- gauge-covariant parallel-transport network -------------------------

def layer_weight_count(cin: int, cout: int) -> int:
    """complex weights of one layer: [9][cout][cin][4][4]"""
    return 9 * cout * cin * 16


def net_weight_count(widths) -> int:
    return sum(layer_weight_count(widths[l], widths[l + 1]) for l in range(len(widths) - 1))


def pt_layer(dims, t_bc, U, cin, cout, W, x, adjoint=False):
    """x: [cin][V][4][3] (or [cout][V][4][3] for the adjoint)."""
    d = _dims(dims)
    v = int(np.prod(d))
    W = _c128(W)
    x = _c128(x)
    out = np.zeros((cin if adjoint else cout, v, 4, 3), dtype=np.complex128)
    fn = load_oracle().orc_pt_layer_adj if adjoint else load_oracle().orc_pt_layer
    fn(_ptr(d), int(t_bc), _ptr(_c128(U)), int(cin), int(cout), _ptr(W), _ptr(x), _ptr(out))
    return out


def pt_net(dims, t_bc, U, widths, W, x, adjoint=False):
    d = _dims(dims)
    v = int(np.prod(d))
    wd = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    nout = wd[0] if adjoint else wd[-1]
    out = np.zeros((nout, v, 4, 3), dtype=np.complex128)
    load_oracle().orc_pt_net(_ptr(d), int(t_bc), _ptr(_c128(U)), len(wd) - 1, _ptr(wd), _ptr(_c128(W)),
                             _ptr(_c128(x)), _ptr(out), 1 if adjoint else 0)
    return out


def pt_loss_grad(dims, t_bc, U, widths, W, r, e):
    """Loss mean |N r - e|^2/|e|^2 and its Wirtinger gradient d/d conj(W)."""
    d = _dims(dims)
    wd = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    W = _c128(W)
    r = _c128(r)
    e = _c128(e)
    grad = np.zeros_like(W)
    loss = load_oracle().orc_pt_loss_grad(_ptr(d), int(t_bc), _ptr(_c128(U)), len(wd) - 1, _ptr(wd), _ptr(W),
                                          int(r.shape[0]), _ptr(r), _ptr(e), _ptr(grad))
    return float(loss), grad


def fcg(dims, t_bc, kappa, mu, U, widths, W, eta, tol, maxit=-1):
    d = _dims(dims)
    wd = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    eta = _c128(eta)
    x = np.zeros_like(eta)
    st = np.zeros(6, dtype=np.float64)
    load_oracle().orc_fcg(_ptr(d), int(t_bc), float(kappa), float(mu), _ptr(_c128(U)), len(wd) - 1, _ptr(wd),
                          _ptr(_c128(W)), _ptr(eta), float(tol), int(maxit), _ptr(x), _ptr(st))
    return x, {"iters": int(st[0]), "resid_normal": st[1], "resid_true": st[2], "converged": bool(st[3]),
               "truncated": bool(st[4]), "fell_back": bool(st[5])}


def fgmres(dims, t_bc, kappa, mu, U, widths, W, eta, tol, m=16, maxit=-1):
    """Restarted FGMRES(m) on M with the network as right preconditioner."""
    d = _dims(dims)
    wd = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    eta = _c128(eta)
    x = np.zeros_like(eta)
    st = np.zeros(5, dtype=np.float64)
    load_oracle().orc_fgmres(_ptr(d), int(t_bc), float(kappa), float(mu), _ptr(_c128(U)), len(wd) - 1, _ptr(wd),
                             _ptr(_c128(W)), _ptr(eta), float(tol), int(m), int(maxit), _ptr(x), _ptr(st))
    return x, {"iters": int(st[0]), "resid": st[1], "resid_true": st[2], "converged": bool(st[3]),
               "truncated": bool(st[4])}
