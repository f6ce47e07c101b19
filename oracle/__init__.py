"""ctypes front-end of the CPU FP64 oracle (oracle/oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg.  The library package never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ECAPACITY, EEMPTY = 0, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O2, single-threaded)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P, I64, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.orc_tau.argtypes = [P, ctypes.c_uint64, P]
        L.orc_apply_ucc.argtypes = [ctypes.c_int, P, P, I64, P, P, I64, D, P, P, I64, P, P, P]
        L.orc_energy.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, I64, P]
        L.orc_h_apply.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, I64, P]
        L.orc_energy_theta.argtypes = [ctypes.c_int, P, P, I64, P, P, I64, D, P, P, ctypes.c_int, P]
        L.orc_energy_and_grad.argtypes = [ctypes.c_int, P, P, I64, P, P, I64, D, P, P, ctypes.c_int, P, P, P]
        L.orc_fd_grad.argtypes = [ctypes.c_int, P, P, I64, P, P, I64, D, P, P, ctypes.c_int, D, P, I64, P]
        L.orc_set_nearcut_window.argtypes = [D]
        L.orc_set_nearcut_window.restype = None
        L.orc_apply_inverse.argtypes = [ctypes.c_int, P, P, I64, P, P, I64, P, P, I64, P]
        L.orc_entropy_trajectory.argtypes = [ctypes.c_int, P, P, I64, P, P, I64, D, P]
        L.orc_live_trajectory.argtypes = [ctypes.c_int, P, P, I64, P, P, I64, D, P]
        L.orc_set_topk.argtypes = [I64, I64]
        L.orc_uncertainty.argtypes = [ctypes.c_int, P, P, I64, P, P, I64, D, D, P, P, I64, P, P, P, I64, P,
                                      P, P, I64, P, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error {code}")
        self.code = code


def _chk(r):
    if r != 0:
        raise OracleError(r)


def _init(dets0, amps0):
    d = np.ascontiguousarray(np.atleast_1d(np.asarray(dets0, dtype=np.uint64)))
    a = np.ascontiguousarray(np.atleast_1d(np.asarray(amps0, dtype=np.float64)))
    return d, a


def set_nearcut_window(rel: float):
    """Relative width of the near-cut window (default 1e-3)."""
    lib().orc_set_nearcut_window(float(rel))


def set_topk(n_max: int, n_cut: int):
    """N_MAX / N_CUT truncation after every factor for later calls (0, 0: off)."""
    _chk(lib().orc_set_topk(int(n_max), int(n_cut)))


def tau(exc4, D):
    e = np.ascontiguousarray(np.asarray(exc4, dtype=np.int8))
    out = ctypes.c_uint64(0)
    s = lib().orc_tau(_p(e), ctypes.c_uint64(int(D)), ctypes.byref(out))
    return s, int(out.value)


def apply_ucc(nq, dets0, amps0, exc, theta, thr=0.0, cap=None):
    """Final state (dets ascending, amplitudes), number of near-cut events
    and det-updates (sum over factors of the live count before the factor)."""
    d, a = _init(dets0, amps0)
    e = np.ascontiguousarray(exc, dtype=np.int8)
    t = np.ascontiguousarray(theta, dtype=np.float64)
    M = e.shape[0]
    cap = cap or max(1 << 16, 4 * len(d))
    while True:
        do = np.empty(cap, np.uint64)
        ao = np.empty(cap, np.float64)
        n = ctypes.c_int64(0)
        nc = ctypes.c_int64(0)
        du = ctypes.c_int64(0)
        r = lib().orc_apply_ucc(nq, _p(d), _p(a), len(d), _p(e), _p(t), M, float(thr), _p(do), _p(ao), cap,
                                ctypes.byref(n), ctypes.byref(nc), ctypes.byref(du))
        if r == ECAPACITY and n.value > cap:
            cap = n.value
            continue
        _chk(r)
        return do[: n.value].copy(), ao[: n.value].copy(), nc.value, du.value


def live_trajectory(nq, dets0, amps0, exc, theta, thr=0.0):
    """Determinants held initially and after each factor: int64 [M+1]."""
    d, a = _init(dets0, amps0)
    e = np.ascontiguousarray(exc, dtype=np.int8)
    t = np.ascontiguousarray(theta, dtype=np.float64)
    M = e.shape[0]
    out = np.zeros(M + 1, np.int64)
    _chk(lib().orc_live_trajectory(nq, _p(d), _p(a), len(d), _p(e), _p(t), M, float(thr), _p(out)))
    return out


def entropy_trajectory(nq, dets0, amps0, exc, theta, thr=0.0):
    """Entropy (Eq. 6) of the initial state and after each factor: [M+1]."""
    d, a = _init(dets0, amps0)
    e = np.ascontiguousarray(exc, dtype=np.int8)
    t = np.ascontiguousarray(theta, dtype=np.float64)
    M = e.shape[0]
    out = np.empty(M + 1, np.float64)
    _chk(lib().orc_entropy_trajectory(nq, _p(d), _p(a), len(d), _p(e), _p(t), M, float(thr), _p(out)))
    return out


def energy(n_orb, h1, h2, dets, amps, mode=1):
    h1 = np.ascontiguousarray(h1, np.float64)
    h2 = np.ascontiguousarray(h2, np.float64)
    d, a = _init(dets, amps)
    E = ctypes.c_double(0)
    _chk(lib().orc_energy(mode, n_orb, _p(h1), _p(h2), _p(d), _p(a), len(d), ctypes.byref(E)))
    return E.value


def h_apply(n_orb, h1, h2, dets, amps, mode=1):
    h1 = np.ascontiguousarray(h1, np.float64)
    h2 = np.ascontiguousarray(h2, np.float64)
    d, a = _init(dets, amps)
    out = np.empty(len(d))
    _chk(lib().orc_h_apply(mode, n_orb, _p(h1), _p(h2), _p(d), _p(a), len(d), _p(out)))
    return out


def energy_theta(nq, dets0, amps0, exc, theta, thr, h1, h2, mode=1):
    d, a = _init(dets0, amps0)
    e = np.ascontiguousarray(exc, np.int8)
    t = np.ascontiguousarray(theta, np.float64)
    h1 = np.ascontiguousarray(h1, np.float64)
    h2 = np.ascontiguousarray(h2, np.float64)
    E = ctypes.c_double(0)
    _chk(lib().orc_energy_theta(nq, _p(d), _p(a), len(d), _p(e), _p(t), e.shape[0], float(thr), _p(h1), _p(h2),
                                mode, ctypes.byref(E)))
    return E.value


def energy_and_grad(nq, dets0, amps0, exc, theta, thr, h1, h2, mode=1):
    """(E, grad[M], near-cut count) with truncation decisions held fixed."""
    d, a = _init(dets0, amps0)
    e = np.ascontiguousarray(exc, np.int8)
    t = np.ascontiguousarray(theta, np.float64)
    h1 = np.ascontiguousarray(h1, np.float64)
    h2 = np.ascontiguousarray(h2, np.float64)
    M = e.shape[0]
    g = np.zeros(M)
    E = ctypes.c_double(0)
    nc = ctypes.c_int64(0)
    _chk(lib().orc_energy_and_grad(nq, _p(d), _p(a), len(d), _p(e), _p(t), M, float(thr), _p(h1), _p(h2), mode,
                                   ctypes.byref(E), _p(g), ctypes.byref(nc)))
    return E.value, g, nc.value


def fd_grad(nq, dets0, amps0, exc, theta, thr, h1, h2, idx, h=1e-5, mode=1):
    d, a = _init(dets0, amps0)
    e = np.ascontiguousarray(exc, np.int8)
    t = np.ascontiguousarray(theta, np.float64)
    h1 = np.ascontiguousarray(h1, np.float64)
    h2 = np.ascontiguousarray(h2, np.float64)
    ix = np.ascontiguousarray(idx, np.int64)
    out = np.empty(len(ix))
    _chk(lib().orc_fd_grad(nq, _p(d), _p(a), len(d), _p(e), _p(t), e.shape[0], float(thr), _p(h1), _p(h2), mode,
                           float(h), _p(ix), len(ix), _p(out)))
    return out


def apply_inverse(nq, dets0, amps0, exc, theta, cap=None):
    d, a = _init(dets0, amps0)
    e = np.ascontiguousarray(exc, np.int8)
    t = np.ascontiguousarray(theta, np.float64)
    cap = cap or max(1 << 16, 4 * len(d))
    do = np.empty(cap, np.uint64)
    ao = np.empty(cap, np.float64)
    n = ctypes.c_int64(0)
    _chk(lib().orc_apply_inverse(nq, _p(d), _p(a), len(d), _p(e), _p(t), e.shape[0], _p(do), _p(ao), cap,
                                 ctypes.byref(n)))
    return do[: n.value].copy(), ao[: n.value].copy()


def uncertainty(nq, dets0, amps0, exc, theta, thr, window=1e-3):
    """Which truncation decisions of the forward circuit may legitimately
    differ in another evaluation whose rounding differs (oracle.cpp,
    orc_uncertainty): a dict with
      nearcut    [(determinant, step)] with ||phi| - thr| <= window * thr
      uncertain  dict determinant -> last step whose decision was uncertain
      delta      dict determinant -> bound on the amplitude difference
      eps        bound on the relative difference of the common scale
    (another run's amplitudes c' satisfy |c'_D - c_D| <= delta[D] + eps |c_D|)."""
    d, a = _init(dets0, amps0)
    e = np.ascontiguousarray(exc, dtype=np.int8)
    t = np.ascontiguousarray(theta, dtype=np.float64)
    M = e.shape[0]
    cap = 1 << 12
    while True:
        nck, ncs = np.empty(cap, np.uint64), np.empty(cap, np.int64)
        unk, uns = np.empty(cap, np.uint64), np.empty(cap, np.int64)
        dlk, dlv = np.empty(cap, np.uint64), np.empty(cap, np.float64)
        nn, un, dn = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
        eps = ctypes.c_double(0)
        r = lib().orc_uncertainty(nq, _p(d), _p(a), len(d), _p(e), _p(t), M, float(thr), float(window), _p(nck),
                                  _p(ncs), cap, ctypes.byref(nn), _p(unk), _p(uns), cap, ctypes.byref(un), _p(dlk),
                                  _p(dlv), cap, ctypes.byref(dn), ctypes.byref(eps))
        if r == ECAPACITY:
            cap = max(nn.value, un.value, dn.value)
            continue
        _chk(r)
        return {
            "nearcut": [(int(k), int(st)) for k, st in zip(nck[: nn.value], ncs[: nn.value])],
            "nearcut_keys": {int(k) for k in nck[: nn.value]},
            "uncertain": {int(k): int(s) for k, s in zip(unk[: un.value], uns[: un.value])},
            "delta": {int(k): float(v) for k, v in zip(dlk[: dn.value], dlv[: dn.value])},
            "eps": eps.value,
        }
