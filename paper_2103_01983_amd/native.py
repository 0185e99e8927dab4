"""ctypes binding of libptrom (C ABI declared in include/ptrom.h).

Argument marshalling only: every computation runs in the HIP library.  Torch
supplies device memory and the current stream.  If the library has not been
built this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libptrom.so")
# launch parameters chosen by ptrom_autotune on an MI355X (loaded by default)
TUNING_PATH = os.path.join(PKG, "tuning_gfx950.txt")

PTROM_OK, PTROM_ENOCONV = 0, 1
BACKWARD_EULER, TRAPEZOID = 0, 1
JAC_PAPER, JAC_EXACT = 0, 1
NEWTON_GMRES, NEWTON_BLOCK = 0, 1

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f32 = ctypes.c_float
_f64 = ctypes.c_double


class NewtonOpts(ctypes.Structure):
    _fields_ = [("newton_tol", _f64), ("max_newton", _i32), ("gmres_restart", _i32),
                ("gmres_maxit", _i32), ("linear_solver", _i32), ("gmres_tol", _f64),
                ("jac_period", _i32), ("pad", _i32)]


class NewtonStats(ctypes.Structure):
    _fields_ = [("newton_iters", _i32), ("krylov_iters", _i32), ("nonconverged_steps", _i32),
                ("pad", _i32), ("max_final_rel_residual", _f64)]


class RomDesc(ctypes.Structure):
    _fields_ = [("M", _i32), ("Mr", _i32), ("ns", _i32), ("jac_mode", _i32),
                ("Nc", _i64), ("nnz", _i64),
                ("Phibar", _vp), ("xbar0", _vp), ("xqt0", _vp), ("Phit", _vp), ("Gt", _vp),
                ("off", _vp), ("ids", _vp), ("A", _vp),
                ("delta", _f64), ("dt", _f64), ("tol", _f64), ("alpha", _f64),
                ("max_iter", _i32), ("pad", _i32), ("ubar", _vp)]


# name -> (restype, argtypes); the full exported surface of ptrom.h
SIGNATURES = {
    "ptrom_version": (ctypes.c_int, []),
    "ptrom_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "ptrom_destroy": (None, [_vp]),
    "ptrom_last_error": (ctypes.c_char_p, [_vp]),
    "ptrom_velocity": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _vp]),
    "ptrom_velocity_noalloc": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _vp]),
    "ptrom_velocity_f64": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f64, _vp, _vp]),
    "ptrom_jvp": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _vp, _vp]),
    "ptrom_block_jacobian": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _vp]),
    "ptrom_velocity_block_jacobian": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _vp, _vp]),
    "ptrom_vjp": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _vp, _vp, _vp]),
    "ptrom_stream_function": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _vp]),
    "ptrom_hamiltonian": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _vp]),
    "ptrom_velocity_points": (ctypes.c_int, [_vp, _i64, _vp, _i64, _vp, _vp, _f32, _vp, _vp]),
    "ptrom_rk4": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _f32, ctypes.c_int, _vp]),
    "ptrom_rk4_f64": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f64, _f64, ctypes.c_int, _vp]),
    "ptrom_implicit": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _f32, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(NewtonOpts), ctypes.POINTER(NewtonStats), _vp]),
    "ptrom_implicit_forced": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _vp, _f32, ctypes.c_int, ctypes.c_int,
                                             ctypes.POINTER(NewtonOpts), ctypes.POINTER(NewtonStats), _vp]),
    "ptrom_velocity_batched": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ptrom_rk4_batched": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp, _f32, ctypes.c_int,
                                         ctypes.c_int, _vp]),
    "ptrom_rk4_fwd_ckpt": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _f32, ctypes.c_int, ctypes.c_int,
                                          _vp, _vp, _vp]),
    "ptrom_rk4_bwd": (ctypes.c_int, [_vp, _i64, _vp, _vp, _f32, _f32, ctypes.c_int, ctypes.c_int,
                                     _vp, _vp, _vp, _vp, _vp]),
    "ptrom_rom_create": (ctypes.c_int, [_vp, ctypes.POINTER(RomDesc), ctypes.POINTER(_vp)]),
    "ptrom_rom_destroy": (None, [_vp]),
    "ptrom_rom_hyperpair": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ptrom_rom_run": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "ptrom_cluster_build": (ctypes.c_int, [_i64, _vp, _vp, _vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_int,
                                           _f64, _f64, _i64, _vp, ctypes.POINTER(_vp)]),
    "ptrom_cluster_sizes": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "ptrom_cluster_fetch": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ptrom_cluster_destroy": (None, [_vp]),
    "ptrom_cluster_members": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), _vp, _vp]),
    "ptrom_rom_set_split": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_uint32]),
    "ptrom_rom_split_plan": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int, _vp]),
    "ptrom_rom_members": (ctypes.c_int, [_vp, _i64, _vp, _vp]),
    "ptrom_rom_reassign": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, _vp]),
    "ptrom_rom_run_batched": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp, _vp]),
    "ptrom_gram_f64": (ctypes.c_int, [_vp, _i64, ctypes.c_int, _vp, _vp, _vp]),
    "ptrom_combine_f64": (ctypes.c_int, [_vp, _i64, ctypes.c_int, _vp, ctypes.c_int, _vp, _vp, _vp]),
    "ptrom_autotune": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "ptrom_load_tuning": (ctypes.c_int, [_vp, ctypes.c_char_p]),
    "ptrom_pair_config": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32)]),
    "ptrom_pair_plan": (ctypes.c_int, [ctypes.c_char_p, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_uint64)]),
}

_lib = None
_lock = threading.Lock()


def lib():
    """Load libptrom.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError("libptrom.so is not built (python -m paper_2103_01983_amd.build)")
                L = ctypes.CDLL(LIB_PATH)
                for name, (res, args) in SIGNATURES.items():
                    fn = getattr(L, name, None)
                    if fn is None:
                        continue
                    fn.restype = res
                    fn.argtypes = args
                _lib = L
    return _lib


class PtromError(RuntimeError):
    pass


_ctxs = {}


def context(device=None) -> int:
    """Per-device library context (created on first use)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                       (device.index if isinstance(device, torch.device) else int(device)))
    idx = dev.index or 0
    if idx not in _ctxs:
        h = _vp()
        rc = lib().ptrom_create(ctypes.byref(h), idx)
        if rc != PTROM_OK:
            raise PtromError("ptrom_create(device=%d) failed with %d" % (idx, rc))
        if os.path.exists(TUNING_PATH) and not os.environ.get("PTROM_TUNE_CACHE"):
            lib().ptrom_load_tuning(h, TUNING_PATH.encode())
        _ctxs[idx] = h
    return _ctxs[idx]


def make_context(device=0, tuning_path=None):
    """A private library context (not the shared per-device one), optionally
    with its own launch table; release with destroy_context."""
    h = _vp()
    rc = lib().ptrom_create(ctypes.byref(h), int(device))
    if rc != PTROM_OK:
        raise PtromError("ptrom_create(device=%d) failed with %d" % (device, rc))
    if tuning_path:
        _check(h, lib().ptrom_load_tuning(h, tuning_path.encode()), "ptrom_load_tuning")
    return h


def destroy_context(h):
    lib().ptrom_destroy(h)


def _check(ctx, rc, what, warn_ok=False):
    if rc == PTROM_OK or (warn_ok and rc == PTROM_ENOCONV):
        return rc
    msg = lib().ptrom_last_error(ctx)
    raise PtromError("%s failed (%d): %s" % (what, rc, (msg or b"").decode()))


def _stream(t: torch.Tensor):
    return _vp(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t, dtype, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a CUDA/HIP tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if numel is not None and t.numel() != numel:
        raise ValueError("%s must have %d elements (got %d)" % (name, numel, t.numel()))
    return _vp(t.data_ptr())


def _n(xy):
    if xy.dim() != 1 or xy.numel() % 2:
        raise ValueError("xy must be a flat [2N] SoA vector")
    return xy.numel() // 2


# --------------------------------------------------------------- pair sums

def velocity(xy, gamma, delta, out=None, ctx=None):
    n = _n(xy)
    out = torch.empty_like(xy) if out is None else out
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_velocity(c, n, _ptr(xy, torch.float32, 2 * n, "xy"),
                                   _ptr(gamma, torch.float32, n, "gamma"), float(delta),
                                   _ptr(out, torch.float32, 2 * n, "out"), _stream(xy)), "ptrom_velocity")
    return out


def velocity_noalloc(xy, gamma, delta, out, ctx=None):
    """ptrom_velocity_noalloc: the velocity into the caller's ``out`` [2N]; the
    library allocates no device memory for it."""
    n = _n(xy)
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_velocity_noalloc(c, n, _ptr(xy, torch.float32, 2 * n, "xy"),
                                           _ptr(gamma, torch.float32, n, "gamma"), float(delta),
                                           _ptr(out, torch.float32, 2 * n, "out"), _stream(xy)),
           "ptrom_velocity_noalloc")
    return out


def velocity_f64(xy, gamma, delta, out=None):
    n = _n(xy)
    out = torch.empty_like(xy) if out is None else out
    c = context(xy.device)
    _check(c, lib().ptrom_velocity_f64(c, n, _ptr(xy, torch.float64, 2 * n, "xy"),
                                       _ptr(gamma, torch.float64, n, "gamma"), float(delta),
                                       _ptr(out, torch.float64, 2 * n, "out"), _stream(xy)),
           "ptrom_velocity_f64")
    return out


def jvp(xy, gamma, delta, v, out=None, ctx=None):
    n = _n(xy)
    out = torch.empty_like(xy) if out is None else out
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_jvp(c, n, _ptr(xy, torch.float32, 2 * n, "xy"), _ptr(gamma, torch.float32, n, "gamma"),
                              float(delta), _ptr(v, torch.float32, 2 * n, "v"),
                              _ptr(out, torch.float32, 2 * n, "out"), _stream(xy)), "ptrom_jvp")
    return out


def block_jacobian(xy, gamma, delta, out=None, ctx=None):
    n = _n(xy)
    out = torch.empty(4 * n, dtype=torch.float32, device=xy.device) if out is None else out
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_block_jacobian(c, n, _ptr(xy, torch.float32, 2 * n, "xy"),
                                         _ptr(gamma, torch.float32, n, "gamma"), float(delta),
                                         _ptr(out, torch.float32, 4 * n, "out"), _stream(xy)),
           "ptrom_block_jacobian")
    return out


def velocity_block_jacobian(xy, gamma, delta, f=None, B=None, ctx=None):
    """Velocity [2N] and self blocks [4N] in one pass; returns (f, B)."""
    n = _n(xy)
    f = torch.empty(2 * n, dtype=torch.float32, device=xy.device) if f is None else f
    B = torch.empty(4 * n, dtype=torch.float32, device=xy.device) if B is None else B
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_velocity_block_jacobian(c, n, _ptr(xy, torch.float32, 2 * n, "xy"),
                                                  _ptr(gamma, torch.float32, n, "gamma"), float(delta),
                                                  _ptr(f, torch.float32, 2 * n, "f"),
                                                  _ptr(B, torch.float32, 4 * n, "B"), _stream(xy)),
           "ptrom_velocity_block_jacobian")
    return f, B


def vjp(xy, gamma, delta, w, gxy=None, ggamma=None, ctx=None):
    n = _n(xy)
    gxy = torch.empty_like(xy) if gxy is None else gxy
    ggamma = torch.empty_like(gamma) if ggamma is None else ggamma
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_vjp(c, n, _ptr(xy, torch.float32, 2 * n, "xy"), _ptr(gamma, torch.float32, n, "gamma"),
                              float(delta), _ptr(w, torch.float32, 2 * n, "w"),
                              _ptr(gxy, torch.float32, 2 * n, "gxy"), _ptr(ggamma, torch.float32, n, "ggamma"),
                              _stream(xy)), "ptrom_vjp")
    return gxy, ggamma


def stream_function(xy, gamma, delta, out=None, ctx=None):
    """psi_i = -(1/4pi) sum_{j!=i} Gamma_j log(|r|^2+delta^2); H = 1/2 sum Gamma_i psi_i."""
    n = _n(xy)
    out = torch.empty_like(gamma) if out is None else out
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_stream_function(c, n, _ptr(xy, torch.float32, 2 * n, "xy"),
                                          _ptr(gamma, torch.float32, n, "gamma"), float(delta),
                                          _ptr(out, torch.float32, n, "psi"), _stream(xy)), "ptrom_stream_function")
    return out


def hamiltonian(xy, gamma, delta, out=None, ctx=None):
    """Regularized Hamiltonian 1/2 sum_i Gamma_i psi_i (ptrom_hamiltonian): a
    one-element FP64 device tensor."""
    n = _n(xy)
    out = torch.empty(1, dtype=torch.float64, device=xy.device) if out is None else out
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_hamiltonian(c, n, _ptr(xy, torch.float32, 2 * n, "xy"),
                                      _ptr(gamma, torch.float32, n, "gamma"), float(delta),
                                      _ptr(out, torch.float64, 1, "H"), _stream(xy)), "ptrom_hamiltonian")
    return out[0]


def velocity_points(points, xy, gamma, delta, out=None):
    """Velocity at arbitrary points [2][nt] (SoA) induced by all bodies."""
    n = _n(xy)
    nt = _n(points)
    out = torch.empty_like(points) if out is None else out
    c = context(xy.device)
    _check(c, lib().ptrom_velocity_points(c, nt, _ptr(points, torch.float32, 2 * nt, "points"), n,
                                          _ptr(xy, torch.float32, 2 * n, "xy"), _ptr(gamma, torch.float32, n, "gamma"),
                                          float(delta), _ptr(out, torch.float32, 2 * nt, "out"), _stream(xy)),
           "ptrom_velocity_points")
    return out


# --------------------------------------------------------------- steppers

def rk4(xy, gamma, delta, dt, nsteps):
    """In place on xy (float32 [2N])."""
    n = _n(xy)
    c = context(xy.device)
    _check(c, lib().ptrom_rk4(c, n, _ptr(xy, torch.float32, 2 * n, "xy"), _ptr(gamma, torch.float32, n, "gamma"),
                              float(delta), float(dt), int(nsteps), _stream(xy)), "ptrom_rk4")
    return xy


def rk4_f64(xy, gamma, delta, dt, nsteps):
    n = _n(xy)
    c = context(xy.device)
    _check(c, lib().ptrom_rk4_f64(c, n, _ptr(xy, torch.float64, 2 * n, "xy"),
                                  _ptr(gamma, torch.float64, n, "gamma"), float(delta), float(dt), int(nsteps),
                                  _stream(xy)), "ptrom_rk4_f64")
    return xy


def implicit(xy, gamma, delta, dt, nsteps, scheme=BACKWARD_EULER, newton_tol=1e-6, max_newton=20,
             gmres_restart=20, gmres_maxit=60, gmres_tol=1e-3, uinf=None, linear_solver=NEWTON_GMRES,
             jac_period=0):
    """In place on xy; returns NewtonStats.  Synchronises the stream.
    ``uinf`` [2N] (device FP32) is an optional background velocity.
    ``linear_solver`` NEWTON_GMRES (exact Jacobian products) or NEWTON_BLOCK
    (the paper's per-body block Jacobian, refreshed per ``jac_period``)."""
    n = _n(xy)
    c = context(xy.device)
    o = NewtonOpts(float(newton_tol), int(max_newton), int(gmres_restart), int(gmres_maxit), int(linear_solver),
                   float(gmres_tol), int(jac_period), 0)
    st = NewtonStats()
    pu = None if uinf is None else _ptr(uinf, torch.float32, 2 * n, "uinf")
    _check(c, lib().ptrom_implicit_forced(c, n, _ptr(xy, torch.float32, 2 * n, "xy"),
                                          _ptr(gamma, torch.float32, n, "gamma"), float(delta), pu, float(dt),
                                          int(nsteps), int(scheme), ctypes.byref(o), ctypes.byref(st), _stream(xy)),
           "ptrom_implicit_forced", warn_ok=True)
    return st


# --------------------------------------------------------------- batched

def _host_i64(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
    return a, a.ctypes.data_as(_vp)


def _host_f32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    return a, a.ctypes.data_as(_vp)


def velocity_batched(offsets, xy, gamma, delta, out=None, ctx=None):
    off, poff = _host_i64(offsets)
    dl, pdl = _host_f32(delta)
    nb = off.size - 1
    tot = int(off[-1])
    out = torch.empty_like(xy) if out is None else out
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_velocity_batched(c, nb, poff, _ptr(xy, torch.float32, 2 * tot, "xy"),
                                           _ptr(gamma, torch.float32, tot, "gamma"), pdl,
                                           _ptr(out, torch.float32, 2 * tot, "out"), _stream(xy)),
           "ptrom_velocity_batched")
    return out


def rk4_batched(offsets, xy, gamma, delta, dt, nsteps, use_graph=True, ctx=None):
    off, poff = _host_i64(offsets)
    dl, pdl = _host_f32(delta)
    nb = off.size - 1
    tot = int(off[-1])
    c = context(xy.device) if ctx is None else ctx
    _check(c, lib().ptrom_rk4_batched(c, nb, poff, _ptr(xy, torch.float32, 2 * tot, "xy"),
                                      _ptr(gamma, torch.float32, tot, "gamma"), pdl, float(dt), int(nsteps),
                                      int(bool(use_graph)), _stream(xy)), "ptrom_rk4_batched")
    return xy


# --------------------------------------------------------------- adjoint

def n_checkpoints(nsteps, every):
    return (nsteps + every - 1) // every


def rk4_fwd_ckpt(xy0, gamma, delta, dt, nsteps, every, ckpt=None, xyT=None):
    n = _n(xy0)
    nck = n_checkpoints(nsteps, every)
    ckpt = torch.empty(max(nck, 1) * 2 * n, dtype=torch.float32, device=xy0.device) if ckpt is None else ckpt
    xyT = torch.empty_like(xy0) if xyT is None else xyT
    c = context(xy0.device)
    _check(c, lib().ptrom_rk4_fwd_ckpt(c, n, _ptr(xy0, torch.float32, 2 * n, "xy0"),
                                       _ptr(gamma, torch.float32, n, "gamma"), float(delta), float(dt),
                                       int(nsteps), int(every), _ptr(ckpt, torch.float32, None, "ckpt"),
                                       _ptr(xyT, torch.float32, 2 * n, "xyT"), _stream(xy0)), "ptrom_rk4_fwd_ckpt")
    return ckpt, xyT


def rk4_bwd(ckpt, gamma, delta, dt, nsteps, every, lamT, ggamma_direct=None, lam0=None, ggamma=None):
    n = gamma.numel()
    lam0 = torch.empty_like(lamT) if lam0 is None else lam0
    ggamma = torch.empty_like(gamma) if ggamma is None else ggamma
    c = context(gamma.device)
    _check(c, lib().ptrom_rk4_bwd(c, n, _ptr(ckpt, torch.float32, None, "ckpt"), _ptr(gamma, torch.float32, n, "gamma"),
                                  float(delta), float(dt), int(nsteps), int(every),
                                  _ptr(lamT, torch.float32, 2 * n, "lamT"),
                                  _ptr(ggamma_direct, torch.float32, n, "ggamma_direct"),
                                  _ptr(lam0, torch.float32, 2 * n, "lam0"), _ptr(ggamma, torch.float32, n, "ggamma"),
                                  _stream(gamma)), "ptrom_rk4_bwd")
    return lam0, ggamma


# --------------------------------------------------------------- online ROM

class Rom:
    """Device-resident online PTROM built from host artifacts (dict as produced
    by the offline training): keys M, Phibar [nd,M], xbar0 [nd], xqt0 [Nc,2],
    Phit [Nc,2,M], Gt [Nc], off [ns+1], ids [nnz], A [Mr,nd], delta, dt."""

    def __init__(self, art, tol=1e-4, max_iter=100, alpha=1.0, jac_mode=JAC_PAPER, device=None):
        c = context(device)
        self._ctx = c
        keep = []

        def d(a, shape=None):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
            keep.append(a)
            return a.ctypes.data_as(_vp)

        def i(a):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.int64))
            keep.append(a)
            return a.ctypes.data_as(_vp)

        off = np.asarray(art["off"], dtype=np.int64)
        ns = off.size - 1
        A = np.asarray(art["A"], dtype=np.float64)
        self.M, self.ns, self.Mr = int(art["M"]), ns, int(A.shape[0])
        if art.get("ubar") is not None and np.asarray(art["ubar"]).size != 2 * ns:
            raise ValueError("ubar must hold the 2 ns sampled rows")
        Nc = int(np.asarray(art["Gt"]).size)
        ids = np.asarray(art["ids"], dtype=np.int64)
        desc = RomDesc(self.M, self.Mr, ns, int(jac_mode), Nc, int(ids.size),
                       d(art["Phibar"]), d(art["xbar0"]), d(np.asarray(art["xqt0"]).reshape(-1)),
                       d(np.asarray(art["Phit"]).reshape(-1)), d(art["Gt"]), i(off), i(ids if ids.size else [0]),
                       d(A), float(art["delta"]), float(art["dt"]), float(tol), float(alpha), int(max_iter), 0,
                       d(art["ubar"]) if art.get("ubar") is not None else None)
        h = _vp()
        _check(c, lib().ptrom_rom_create(c, ctypes.byref(desc), ctypes.byref(h)), "ptrom_rom_create")
        self._h = h
        self.Nc = Nc
        if "mem_off" in art and "n" in art:
            self.set_members(art["mem_off"], art["mem_ids"], art["n"])

    def close(self):
        if getattr(self, "_h", None):
            lib().ptrom_rom_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def hyperpair(self, xhat, xbar_prev, fbar_prev):
        nd = 2 * self.ns
        dev = xhat.device
        xbar = torch.empty(nd, dtype=torch.float64, device=dev)
        fbar = torch.empty_like(xbar)
        rbar = torch.empty_like(xbar)
        C = torch.empty(nd * self.M, dtype=torch.float64, device=dev)
        _check(self._ctx, lib().ptrom_rom_hyperpair(self._h, _ptr(xhat, torch.float64, self.M, "xhat"),
                                                    _ptr(xbar_prev, torch.float64, nd, "xbar_prev"),
                                                    _ptr(fbar_prev, torch.float64, nd, "fbar_prev"),
                                                    _ptr(xbar, torch.float64, nd, "xbar"),
                                                    _ptr(fbar, torch.float64, nd, "fbar"),
                                                    _ptr(rbar, torch.float64, nd, "rbar"),
                                                    _ptr(C, torch.float64, nd * self.M, "C"), _stream(xhat)),
               "ptrom_rom_hyperpair")
        return xbar, fbar, rbar, C.view(nd, self.M)

    def run(self, nsteps, xhat, hist=None, iters=None):
        _check(self._ctx, lib().ptrom_rom_run(self._h, int(nsteps), _ptr(xhat, torch.float64, self.M, "xhat"),
                                              _ptr(hist, torch.float64, nsteps * self.M, "hist"),
                                              _ptr(iters, torch.int32, nsteps, "iters"), _stream(xhat)),
               "ptrom_rom_run")
        return xhat

    def set_split(self, workgroups, max_polls=0):
        """Workgroups per query of the small-basis paper-Jacobian runs (0 automatic, 1 none);
        max_polls: failed barrier checks before a split run aborts (0 default)."""
        _check(self._ctx, lib().ptrom_rom_set_split(self._h, int(workgroups), int(max_polls)),
               "ptrom_rom_set_split")

    def split_plan(self, nsteps, batched_nq=0):
        """Workgroups per query that run (batched_nq = 0) or run_batched would use."""
        w = ctypes.c_int32(0)
        _check(self._ctx, lib().ptrom_rom_split_plan(self._h, int(batched_nq), int(nsteps), ctypes.byref(w)),
               "ptrom_rom_split_plan")
        return int(w.value)

    def set_members(self, mem_off, mem_ids, n):
        """Bodies of each surrogate (CSR, host), for parametric queries."""
        mem_off = np.ascontiguousarray(mem_off, dtype=np.int64)
        mem_ids = np.ascontiguousarray(mem_ids, dtype=np.int64)
        if mem_off.size != self.Nc + 1:
            raise ValueError("mem_off must have Nc + 1 entries")
        self.n = int(n)
        _check(self._ctx, lib().ptrom_rom_members(self._h, self.n, mem_off.ctypes.data_as(_vp),
                                                  mem_ids.ctypes.data_as(_vp) if mem_ids.size else None),
               "ptrom_rom_members")

    def reassign(self, gamma_q):
        """Clustered circulations for parameters gamma_q (device FP32 [nq, n]): [nq, Nc]."""
        nq = gamma_q.shape[0]
        out = torch.empty((nq, self.Nc), dtype=torch.float32, device=gamma_q.device)
        _check(self._ctx, lib().ptrom_rom_reassign(self._h, int(nq), _ptr(gamma_q, torch.float32, nq * self.n, "gamma_q"),
                                                   _ptr(out, torch.float32, nq * self.Nc, "gt_q"), _stream(gamma_q)),
               "ptrom_rom_reassign")
        return out

    def run_batched(self, gt_q, nsteps, xhat, hist=None, iters=None):
        """nq online runs in one launch: gt_q [nq, Nc] FP32, xhat [nq, M] FP64 (in place)."""
        nq = gt_q.shape[0]
        _check(self._ctx, lib().ptrom_rom_run_batched(
            self._h, int(nq), _ptr(gt_q, torch.float32, nq * self.Nc, "gt_q"), int(nsteps),
            _ptr(xhat, torch.float64, nq * self.M, "xhat"), _ptr(hist, torch.float64, nq * nsteps * self.M, "hist"),
            _ptr(iters, torch.int32, nq * nsteps, "iters"), _stream(gt_q)), "ptrom_rom_run_batched")
        return xhat


# --------------------------------------------------------------- offline helpers

NEIGHBOR, BARNES_HUT = 0, 1


def cluster_build(wpts, xy0, phi, gamma, max_level, pc, targets, criterion=NEIGHBOR, theta=0.0):
    """Host quadtree + source clustering (native).  Returns dict with
    xqt0 [Nc,2], Phit [Nc,2,M], Gt [Nc], off [nt+1], ids [nnz], keys [Nc]."""
    wpts = np.ascontiguousarray(wpts, dtype=np.float64)
    xy0 = np.ascontiguousarray(xy0, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    n = gamma.size
    M = phi.shape[1]
    if wpts.shape != (n, 2) or xy0.size != 2 * n or phi.shape[0] != 2 * n:
        raise ValueError("inconsistent shapes")
    h = _vp()
    L = lib()
    rc = L.ptrom_cluster_build(n, wpts.ctypes.data_as(_vp), xy0.ctypes.data_as(_vp), phi.ctypes.data_as(_vp), M,
                               gamma.ctypes.data_as(_vp), int(max_level), int(criterion), float(pc), float(theta),
                               targets.size, targets.ctypes.data_as(_vp), ctypes.byref(h))
    if rc != PTROM_OK:
        raise PtromError("ptrom_cluster_build failed (%d)" % rc)
    try:
        nc, nnz = _i64(), _i64()
        L.ptrom_cluster_sizes(h, ctypes.byref(nc), ctypes.byref(nnz))
        nc, nnz = nc.value, nnz.value
        out = dict(xqt0=np.empty((nc, 2)), Phit=np.empty((nc, 2, M)), Gt=np.empty(nc),
                   off=np.empty(targets.size + 1, np.int64), ids=np.empty(max(nnz, 1), np.int64),
                   keys=np.empty(max(nc, 1), np.int64))
        L.ptrom_cluster_fetch(h, out["xqt0"].ctypes.data_as(_vp), out["Phit"].ctypes.data_as(_vp),
                              out["Gt"].ctypes.data_as(_vp), out["off"].ctypes.data_as(_vp),
                              out["ids"].ctypes.data_as(_vp), out["keys"].ctypes.data_as(_vp))
        out["ids"] = out["ids"][:nnz]
        out["keys"] = out["keys"][:nc]
        nmem = _i64()
        L.ptrom_cluster_members(h, ctypes.byref(nmem), None, None)
        out["mem_off"] = np.empty(nc + 1, np.int64)
        out["mem_ids"] = np.empty(max(nmem.value, 1), np.int64)
        L.ptrom_cluster_members(h, ctypes.byref(nmem), out["mem_off"].ctypes.data_as(_vp),
                                out["mem_ids"].ctypes.data_as(_vp))
        out["mem_ids"] = out["mem_ids"][:nmem.value]
        return out
    finally:
        L.ptrom_cluster_destroy(h)


def gram_f64(X, out=None):
    """G = X X^T for a device FP64 [k, nd] tensor."""
    k, nd = X.shape
    out = torch.empty((k, k), dtype=torch.float64, device=X.device) if out is None else out
    c = context(X.device)
    _check(c, lib().ptrom_gram_f64(c, nd, k, _ptr(X, torch.float64, k * nd, "X"),
                                   _ptr(out, torch.float64, k * k, "G"), _stream(X)), "ptrom_gram_f64")
    return out


def combine_f64(X, T, out=None):
    """Y = T^T X for device FP64 X [k, nd], T [k, M]; returns Y [M, nd]."""
    k, nd = X.shape
    M = T.shape[1]
    out = torch.empty((M, nd), dtype=torch.float64, device=X.device) if out is None else out
    c = context(X.device)
    _check(c, lib().ptrom_combine_f64(c, nd, k, _ptr(X, torch.float64, k * nd, "X"), M,
                                      _ptr(T, torch.float64, k * M, "T"), _ptr(out, torch.float64, M * nd, "Y"),
                                      _stream(X)), "ptrom_combine_f64")
    return out


# --------------------------------------------------------------- tuning

def autotune(cache_path=None, device=None):
    c = context(device)
    _check(c, lib().ptrom_autotune(c, cache_path.encode() if cache_path else None), "ptrom_autotune")


def load_tuning(cache_path, device=None):
    c = context(device)
    _check(c, lib().ptrom_load_tuning(c, cache_path.encode()), "ptrom_load_tuning")


PAIR_OPS = {"velocity": 0, "block_jacobian": 1, "jvp": 2, "vjp": 3, "stream_function": 4,
            "velocity_block_jacobian": 5}
# tuning-table entry of the batched velocity launch (ptrom_pair_config key 6)
BATCHED_OP = ("batched_velocity", 6)


def pair_config(op, n, device=None, ctx=None):
    """The launch the library picks for pair operation ``op`` (a name of
    PAIR_OPS) at n bodies: dict(staging, k, waves_per_simd, sym, splits)."""
    c = context(device) if ctx is None else ctx
    out = (ctypes.c_int32 * 5)()
    code = BATCHED_OP[1] if op == BATCHED_OP[0] else PAIR_OPS[op]
    _check(c, lib().ptrom_pair_config(c, code, int(n), out), "ptrom_pair_config")
    return dict(staging=int(out[0]), k=int(out[1]), waves_per_simd=int(out[2]), sym=int(out[3]),
                splits=int(out[4]))


def pair_plan(op, n, num_cus=256, device_bytes=288 * 10**9, tuning_path=TUNING_PATH):
    """The launch and workspace (bytes) a device with ``num_cus`` compute units
    and ``device_bytes`` of memory would use for ``op`` at n bodies (host only,
    no GPU needed): dict(staging, k, waves_per_simd, sym, splits, ws_bytes)."""
    out = (ctypes.c_int32 * 5)()
    ws = ctypes.c_uint64()
    rc = lib().ptrom_pair_plan(tuning_path.encode() if tuning_path else None, int(num_cus), int(device_bytes),
                               PAIR_OPS[op], int(n), out, ctypes.byref(ws))
    if rc != PTROM_OK:
        raise PtromError("ptrom_pair_plan failed (%d)" % rc)
    return dict(staging=int(out[0]), k=int(out[1]), waves_per_simd=int(out[2]), sym=int(out[3]),
                splits=int(out[4]), ws_bytes=int(ws.value))
