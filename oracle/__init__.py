"""FP64 CPU oracle for the regularized 2D Biot-Savart hot path of the
projection-tree ROM (arXiv 2103.01983).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library: the numerical kernels live in ``oracle.c`` (plain double loops,
OpenMP over independent targets) and the offline pipeline in ``offline.py``
(NumPy, FP64).

Every array is float64 NumPy.  State vectors use the paper's layout
``x = [chi_1..chi_N, psi_1..psi_N]`` (problem formulation, state vector).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (x86-64 baseline ISA,
    so no FMA contraction; OpenMP over targets)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class NewtonStats(ctypes.Structure):
    _fields_ = [
        ("newton_iters", ctypes.c_int32),
        ("krylov_iters", ctypes.c_int32),
        ("nonconverged_steps", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("max_final_rel_residual", ctypes.c_double),
    ]


class _Rom(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("Mr", ctypes.c_int32), ("ns", ctypes.c_int32), ("jac_mode", ctypes.c_int32),
        ("Nc", ctypes.c_int64),
        ("Phibar", _dp), ("xbar0", _dp), ("xqt0", _dp), ("Phit", _dp), ("Gt", _dp), ("A", _dp),
        ("off", _i64p), ("ids", _i64p),
        ("delta", ctypes.c_double), ("dt", ctypes.c_double),
        ("ubar", _dp),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        i64, dbl, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        L.or_velocity.argtypes = [i64, _dp, _dp, dbl, _dp]
        L.or_velocity_at.argtypes = [i64, _dp, _dp, dbl, i64, _i64p, _dp]
        L.or_jvp.argtypes = [i64, _dp, _dp, dbl, _dp, _dp]
        L.or_jvp_at.argtypes = [i64, _dp, _dp, dbl, _dp, i64, _i64p, _dp]
        L.or_block_jacobian.argtypes = [i64, _dp, _dp, dbl, _dp]
        L.or_vjp.argtypes = [i64, _dp, _dp, dbl, _dp, _dp, _dp]
        L.or_vjp_at.argtypes = [i64, _dp, _dp, dbl, _dp, i64, _i64p, _dp, _dp]
        L.or_hamiltonian.argtypes = [i64, _dp, _dp, dbl]
        L.or_hamiltonian.restype = dbl
        L.or_stream_function.argtypes = [i64, _dp, _dp, dbl, _dp]
        L.or_stream_function_at.argtypes = [i64, _dp, _dp, dbl, i64, _i64p, _dp]
        L.or_velocity_points.argtypes = [i64, _dp, i64, _dp, _dp, dbl, _dp]
        L.or_rk4.argtypes = [i64, _dp, _dp, dbl, dbl, i32]
        L.or_implicit.argtypes = [i64, _dp, _dp, dbl, dbl, i32, i32, dbl, i32, dbl, i32, i32,
                                  ctypes.POINTER(NewtonStats)]
        L.or_implicit_forced.argtypes = [i64, _dp, _dp, dbl, _dp, dbl, i32, i32, dbl, i32, dbl, i32, i32,
                                         ctypes.POINTER(NewtonStats)]
        L.or_block_jacobian_at.argtypes = [i64, _dp, _dp, dbl, i64, _i64p, _dp]
        L.or_implicit_block.argtypes = [i64, _dp, _dp, dbl, _dp, dbl, i32, i32, dbl, i32, i32,
                                        ctypes.POINTER(NewtonStats)]
        L.or_rk4_adjoint.argtypes = [i64, _dp, _dp, dbl, dbl, i32, _dp, _dp, _dp, _dp, _dp]
        L.or_lstsq.argtypes = [i32, i32, _dp, _dp, _dp]
        L.or_rom_hyperpair.argtypes = [ctypes.POINTER(_Rom), _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.or_set_threads.argtypes = [i32]
        L.or_set_threads.restype = i32
        L.or_rom_run.argtypes = [ctypes.POINTER(_Rom), dbl, dbl, i32, i32, _dp, _dp, _i32p, _dp, i64, _i64p]
    return _lib


def _d(a):
    """Contiguous float64 copy-or-view and its pointer."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_i64p)


def _n(xy):
    xy = np.asarray(xy)
    assert xy.ndim == 1 and xy.size % 2 == 0
    return xy.size // 2


# ---------------------------------------------------------------------------
# pair sum and derivatives
# ---------------------------------------------------------------------------

def velocity(xy, gamma, delta):
    """f_i = sum_{j!=i} Gamma_j/(2pi) (-r_y, r_x)/(|r|^2+delta^2), r = x_i - x_j."""
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma)
    f = np.empty(2 * n)
    lib().or_velocity(n, pxy, pg, float(delta), f.ctypes.data_as(_dp))
    return f


def velocity_at(xy, gamma, delta, idx):
    """Velocity at the targets ``idx`` only; returns [2][len(idx)] flattened."""
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma); idx, pi = _i(idx)
    out = np.empty(2 * idx.size)
    lib().or_velocity_at(n, pxy, pg, float(delta), idx.size, pi, out.ctypes.data_as(_dp))
    return out


def jvp(xy, gamma, delta, v):
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma); v, pv = _d(v)
    out = np.empty(2 * n)
    lib().or_jvp(n, pxy, pg, float(delta), pv, out.ctypes.data_as(_dp))
    return out


def jvp_at(xy, gamma, delta, v, idx):
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma); v, pv = _d(v); idx, pi = _i(idx)
    out = np.empty(2 * idx.size)
    lib().or_jvp_at(n, pxy, pg, float(delta), pv, idx.size, pi, out.ctypes.data_as(_dp))
    return out


def block_jacobian_at(xy, gamma, delta, idx):
    """The 2x2 blocks of the targets ``idx`` only; returns [4][len(idx)] flattened."""
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma); idx, pi = _i(idx)
    out = np.empty(4 * idx.size)
    lib().or_block_jacobian_at(n, pxy, pg, float(delta), idx.size, pi, out.ctypes.data_as(_dp))
    return out


def block_jacobian(xy, gamma, delta):
    """Per-target 2x2 blocks of df/dx; returns [4][N] (B00, B01, B10, B11)."""
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma)
    out = np.empty(4 * n)
    lib().or_block_jacobian(n, pxy, pg, float(delta), out.ctypes.data_as(_dp))
    return out


def vjp(xy, gamma, delta, w):
    """Returns (J^T w [2N], d(w.f)/dGamma [N])."""
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma); w, pw = _d(w)
    gx = np.empty(2 * n); gg = np.empty(n)
    lib().or_vjp(n, pxy, pg, float(delta), pw, gx.ctypes.data_as(_dp), gg.ctypes.data_as(_dp))
    return gx, gg


def vjp_at(xy, gamma, delta, w, idx):
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma); w, pw = _d(w); idx, pi = _i(idx)
    gx = np.empty(2 * idx.size); gg = np.empty(idx.size)
    lib().or_vjp_at(n, pxy, pg, float(delta), pw, idx.size, pi, gx.ctypes.data_as(_dp), gg.ctypes.data_as(_dp))
    return gx, gg


def hamiltonian(xy, gamma, delta):
    """Regularized Hamiltonian -(1/4pi) sum_{i!=j} G_i G_j log(|r|^2+delta^2)/2."""
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma)
    return lib().or_hamiltonian(n, pxy, pg, float(delta))


def stream_function(xy, gamma, delta):
    """psi_i = -(1/4pi) sum_{j!=i} Gamma_j log(|r|^2+delta^2); H = 1/2 sum Gamma_i psi_i."""
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma)
    out = np.empty(n)
    lib().or_stream_function(n, pxy, pg, float(delta), out.ctypes.data_as(_dp))
    return out


def stream_function_at(xy, gamma, delta, idx):
    """psi at the targets ``idx`` only."""
    n = _n(xy)
    xy, pxy = _d(xy); g, pg = _d(gamma); idx, pi = _i(idx)
    out = np.empty(idx.size)
    lib().or_stream_function_at(n, pxy, pg, float(delta), idx.size, pi, out.ctypes.data_as(_dp))
    return out


def velocity_points(points, xy, gamma, delta):
    """Velocity at arbitrary points [2][nt] (SoA) induced by all bodies."""
    n = _n(xy)
    p, pp = _d(points); xy, pxy = _d(xy); g, pg = _d(gamma)
    nt = p.size // 2
    out = np.empty(2 * nt)
    lib().or_velocity_points(nt, pp, n, pxy, pg, float(delta), out.ctypes.data_as(_dp))
    return out


# ---------------------------------------------------------------------------
# time steppers
# ---------------------------------------------------------------------------

def set_threads(n):
    """Thread count of the oracle's OpenMP loops; returns the previous one."""
    return int(lib().or_set_threads(int(n)))


def rk4(xy, gamma, delta, dt, nsteps):
    n = _n(xy)
    x = np.array(xy, dtype=np.float64, copy=True)
    g, pg = _d(gamma)
    rc = lib().or_rk4(n, x.ctypes.data_as(_dp), pg, float(delta), float(dt), int(nsteps))
    assert rc == 0
    return x


BE, TRAPEZOID = 0, 1


def implicit(xy, gamma, delta, dt, nsteps, scheme=BE, newton_tol=1e-12, max_newton=50,
             gmres_tol=1e-14, gmres_restart=40, gmres_maxit=400, u=None):
    """k=1 implicit linear multistep steps (backward Euler or trapezoid) solved by
    Newton-GMRES with the exact Jacobian product; ``u`` [2N] is an optional
    background velocity (dx/dt = f(x) + u).  Returns (x, NewtonStats)."""
    n = _n(xy)
    x = np.array(xy, dtype=np.float64, copy=True)
    g, pg = _d(gamma)
    pu = None
    if u is not None:
        ua, pu = _d(u)
        assert ua.size == 2 * n
    st = NewtonStats()
    lib().or_implicit_forced(n, x.ctypes.data_as(_dp), pg, float(delta), pu, float(dt), int(nsteps), int(scheme),
                             float(newton_tol), int(max_newton), float(gmres_tol), int(gmres_restart),
                             int(gmres_maxit), ctypes.byref(st))
    return x, st


def implicit_block(xy, gamma, delta, dt, nsteps, scheme=BE, newton_tol=1e-12, max_newton=100, jac_period=0,
                   u=None):
    """The paper's FOM solver: k=1 implicit steps by inexact Newton with the
    block-diagonal kernel Jacobian (per-body 2x2 solves), evaluated at every
    iterate (jac_period 0) or at the start of every jac_period-th step.
    Returns (x, NewtonStats)."""
    n = _n(xy)
    x = np.array(xy, dtype=np.float64, copy=True)
    g, pg = _d(gamma)
    pu = None
    if u is not None:
        ua, pu = _d(u)
        assert ua.size == 2 * n
    st = NewtonStats()
    lib().or_implicit_block(n, x.ctypes.data_as(_dp), pg, float(delta), pu, float(dt), int(nsteps), int(scheme),
                            float(newton_tol), int(max_newton), int(jac_period), ctypes.byref(st))
    return x, st


def rk4_adjoint(xy0, gamma, delta, dt, nsteps, lamT, gg_direct=None):
    """Discrete adjoint of ``nsteps`` RK4 steps.  Given lamT = dQ/dx(T) and the
    direct Gamma-partial of Q, returns (x(T), dQ/dx(0), dQ/dGamma)."""
    n = _n(xy0)
    x0, px = _d(xy0); g, pg = _d(gamma); lam, pl = _d(lamT)
    if gg_direct is None:
        pgd = None
    else:
        gd, pgd = _d(gg_direct)
    xT = np.empty(2 * n); lam0 = np.empty(2 * n); gg = np.empty(n)
    rc = lib().or_rk4_adjoint(n, px, pg, float(delta), float(dt), int(nsteps), pl, pgd,
                              xT.ctypes.data_as(_dp), lam0.ctypes.data_as(_dp), gg.ctypes.data_as(_dp))
    assert rc == 0
    return xT, lam0, gg


def lstsq(G, b):
    """min |G x - b| by the oracle's Householder QR (G: m x n, m >= n)."""
    G, pG = _d(G); b, pb = _d(b)
    m, n = G.shape
    x = np.empty(n)
    lib().or_lstsq(m, n, pG, pb, x.ctypes.data_as(_dp))
    return x


# ---------------------------------------------------------------------------
# online PTROM
# ---------------------------------------------------------------------------

class Rom:
    """Online PTROM (Gauss-Newton around HyperPair) on fixed offline artifacts.

    ``art`` is a dict with keys M, Mr, sample (body ids), Phibar [nd,M],
    xbar0 [nd], xqt0 [Nc,2], Phit [Nc,2,M], Gt [Nc], off [ns+1], ids [nnz],
    A [Mr,nd] or None (identity), delta, dt.  jac_mode 0 = the paper's
    inexact Jacobian, 1 = exact.
    """

    def __init__(self, art, jac_mode=0):
        self._keep = {}
        def d(key, arr):
            a, p = _d(arr)
            self._keep[key] = a
            return p
        def i(key, arr):
            a, p = _i(arr)
            self._keep[key] = a
            return p
        ns = int(len(art["off"]) - 1)
        M = int(art["M"])
        nd = 2 * ns
        A = art.get("A")
        self.M, self.ns = M, ns
        Nc = int(np.asarray(art["Gt"]).size)
        r = _Rom()
        r.M, r.ns, r.jac_mode = M, ns, int(jac_mode)
        r.Mr = int(np.asarray(A).shape[0]) if A is not None else nd
        r.Nc = Nc
        r.Phibar = d("Phibar", np.asarray(art["Phibar"]).reshape(nd, M))
        r.xbar0 = d("xbar0", art["xbar0"])
        r.xqt0 = d("xqt0", np.asarray(art["xqt0"]).reshape(-1) if Nc else np.zeros(2))
        r.Phit = d("Phit", np.asarray(art["Phit"]).reshape(-1) if Nc else np.zeros(2 * M))
        r.Gt = d("Gt", art["Gt"] if Nc else np.zeros(1))
        r.A = d("A", A) if A is not None else None
        r.off = i("off", art["off"])
        r.ids = i("ids", art["ids"] if len(art["ids"]) else np.zeros(1, np.int64))
        r.delta = float(art["delta"])
        r.dt = float(art["dt"])
        ub = art.get("ubar")
        r.ubar = d("ubar", np.asarray(ub, dtype=np.float64).reshape(nd)) if ub is not None else None
        self._r = r

    def hyperpair(self, xhat, xbar_prev, fbar_prev):
        """One HyperPair evaluation: returns (xbar, fbar, rbar, C)."""
        nd, M = 2 * self.ns, self.M
        xh, p1 = _d(xhat); xp, p2 = _d(xbar_prev); fp, p3 = _d(fbar_prev)
        xbar = np.empty(nd); fbar = np.empty(nd); rbar = np.empty(nd); C = np.empty((nd, M))
        lib().or_rom_hyperpair(ctypes.byref(self._r), p1, p2, p3, xbar.ctypes.data_as(_dp),
                               fbar.ctypes.data_as(_dp), rbar.ctypes.data_as(_dp), C.ctypes.data_as(_dp))
        return xbar, fbar, rbar, C

    def run(self, nsteps, xhat0=None, tol=1e-4, max_iter=100, alpha=1.0, resid_cap=0):
        """Returns dict(xhat, hist [nsteps,M], iters [nsteps], status, resid [k,nd])."""
        M, nd = self.M, 2 * self.ns
        xh = np.zeros(M) if xhat0 is None else np.array(xhat0, dtype=np.float64, copy=True)
        hist = np.empty((nsteps, M)); iters = np.empty(nsteps, dtype=np.int32)
        resid = np.empty((max(resid_cap, 1), nd)) if resid_cap else None
        cnt = ctypes.c_int64(0)
        st = lib().or_rom_run(ctypes.byref(self._r), float(alpha), float(tol), int(max_iter), int(nsteps),
                              xh.ctypes.data_as(_dp), hist.ctypes.data_as(_dp), iters.ctypes.data_as(_i32p),
                              resid.ctypes.data_as(_dp) if resid is not None else None, int(resid_cap),
                              ctypes.byref(cnt))
        out = dict(xhat=xh, hist=hist, iters=iters, status=st, nresid=cnt.value)
        if resid is not None:
            out["resid"] = resid[: min(cnt.value, resid_cap)]
        return out
