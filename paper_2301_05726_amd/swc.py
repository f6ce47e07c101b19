"""Python binding of libswc.so (C ABI in include/swc.h).

Argument marshalling only: every step of the circuit, energy and gradient
runs in the HIP library.  PyTorch provides the device workspace and the
stream.  There is no fallback: if the library is not built, or no GPU is
present, the calls raise.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libswc.so")

OK, EINVAL, ECAPACITY, EEMPTY, EDEVICE, ESTATE = 0, -1, -2, -3, -4, -5
FP64, FP32 = 0, 1

EXPORTS = [
    "swc_workspace_bytes", "swc_create", "swc_build_state", "swc_apply_ucc", "swc_energy",
    "swc_energy_and_grad", "swc_get_state", "swc_get_stats", "swc_strerror", "swc_last_error",
    "swc_destroy", "swc_validate_excitations", "swc_factor_masks", "swc_checkpoint_bytes",
    "swc_set_checkpoints", "swc_track_entropy", "swc_get_entropy", "swc_set_topk", "swc_set_sigma_scratch",
    "swc_track_live", "swc_get_live_counts", "swc_energy_noalloc",
]

NOALLOC_MAX_DETS = 65536  # SWC_NOALLOC_MAX_DETS


class SwcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"swc error {code}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_live", ctypes.c_int64), ("det_updates", ctypes.c_int64), ("pair_updates", ctypes.c_int64),
        ("inserts", ctypes.c_int64), ("pruned", ctypes.c_int64), ("log_records", ctypes.c_int64),
        ("table_slots", ctypes.c_int64), ("slots_used", ctypes.c_int64),
        ("fwd_ms", ctypes.c_double), ("energy_ms", ctypes.c_double), ("rev_ms", ctypes.c_double),
        ("rotate_kernel_ms", ctypes.c_double), ("rotate_launches", ctypes.c_int64),
        ("reverse_kernel_ms", ctypes.c_double), ("reverse_launches", ctypes.c_int64),
        ("sigma_kernel_ms", ctypes.c_double), ("partner_hits", ctypes.c_int64),
        ("rehashes", ctypes.c_int64), ("compactions", ctypes.c_int64), ("checkpoints", ctypes.c_int64),
        ("sigma_partitions", ctypes.c_int64),
        ("shrinks", ctypes.c_int64),
        ("fwd_slots_scanned", ctypes.c_int64),
        ("rev_slots_scanned", ctypes.c_int64),
        ("grad_calls", ctypes.c_int64), ("fwd_ms_total", ctypes.c_double), ("rev_ms_total", ctypes.c_double),
        ("sigma_kernel_ms_total", ctypes.c_double),
        ("kernel_builds", ctypes.c_int64),
    ]


# sweep kernel builds (Stats.kernel_builds bits)
BUILD_FWD, BUILD_FWD_ENT, BUILD_FWD2, BUILD_FWD2_PRE = 1, 4, 8, 16
BUILD_REV, BUILD_REV2, BUILD_REV2_PRE, BUILD_PERSISTENT = 32, 64, 128, 256
BUILD_FWD_HO, BUILD_FWD_PF, BUILD_REV_PF = 512, 1024, 2048


_lib = None

# Contexts not yet closed.  They are destroyed by an exit hook that runs
# before the interpreter finalises (torch and the HIP runtime still intact),
# so no HIP call is left for object finalisers during interpreter shutdown.
_open_solvers: "weakref.WeakSet[Solver]" = weakref.WeakSet()


@atexit.register
def _close_open_solvers():
    for s in list(_open_solvers):
        s.close()


def lib():
    """Load libswc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2301_05726_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I, I64, U64, D, SZ = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_double, ctypes.c_size_t)
        L.swc_workspace_bytes.argtypes = [I, U64, I, I, I64, U64]
        L.swc_workspace_bytes.restype = SZ
        L.swc_create.argtypes = [ctypes.POINTER(P), I, I, I, U64, I, I, I64, U64, P, SZ, P]
        L.swc_build_state.argtypes = [P, P, P, I64]
        L.swc_apply_ucc.argtypes = [P, P, P, I64, D]
        L.swc_energy.argtypes = [P, P, P, P]
        L.swc_energy_and_grad.argtypes = [P, P, P, I64, D, P, P, P, P]
        L.swc_get_state.argtypes = [P, I, P, P, I64, ctypes.POINTER(I64)]
        L.swc_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
        L.swc_strerror.argtypes = [I]
        L.swc_strerror.restype = ctypes.c_char_p
        L.swc_last_error.argtypes = []
        L.swc_last_error.restype = ctypes.c_char_p
        L.swc_destroy.argtypes = [P]
        L.swc_destroy.restype = None
        L.swc_validate_excitations.argtypes = [I, P, I64]
        L.swc_factor_masks.argtypes = [I, P, I64, P]
        L.swc_checkpoint_bytes.argtypes = [I, I, I64, I64, U64]
        L.swc_checkpoint_bytes.restype = SZ
        L.swc_set_checkpoints.argtypes = [P, I64, U64, P, SZ]
        L.swc_track_entropy.argtypes = [P, I]
        L.swc_get_entropy.argtypes = [P, I, P, I64]
        L.swc_get_live_counts.argtypes = [P, I, P, I64]
        L.swc_track_live.argtypes = [P, I]
        L.swc_set_topk.argtypes = [P, U64, U64]
        L.swc_set_sigma_scratch.argtypes = [P, P, SZ, I]
        L.swc_energy_noalloc.argtypes = [I, P, P, I64, P, P, P, P]
        _lib = L
    return _lib


def _chk(code: int):
    if code != 0:
        raise SwcError(code, lib().swc_last_error().decode())


def _exc_array(exc) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(exc, dtype=np.int8).reshape(-1, 4))
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def validate_excitations(n_qubits: int, exc) -> int:
    """Host-only check (no GPU): 0 or the negative error code."""
    e = _exc_array(exc)
    return lib().swc_validate_excitations(n_qubits, _ptr(e), e.shape[0])


def factor_masks(n_qubits: int, exc) -> np.ndarray:
    """Host-only: per factor (occupied mask, virtual mask, sign mask)."""
    e = _exc_array(exc)
    out = np.zeros((e.shape[0], 3), dtype=np.uint64)
    _chk(lib().swc_factor_masks(n_qubits, _ptr(e), e.shape[0], _ptr(out)))
    return out


def energy_noalloc(n_qubits: int, dets: torch.Tensor, amps: torch.Tensor, h1: torch.Tensor, h2: torch.Tensor,
                   E: torch.Tensor, stream=None) -> None:
    """swc_energy_noalloc: E[0] = <Psi|H|Psi>/<Psi|Psi> of the state (dets,
    amps) with no device allocation by the library.  Every argument is a
    contiguous tensor on the device the call runs on (dets int64 holding the
    64-bit determinants, amps/h1/h2/E float64); the caller allocates them."""
    for name, t, dt in (("dets", dets, torch.int64), ("amps", amps, torch.float64), ("h1", h1, torch.float64),
                        ("h2", h2, torch.float64), ("E", E, torch.float64)):
        if not (t.is_cuda and t.is_contiguous() and t.dtype == dt):
            raise ValueError(f"{name} must be a contiguous {dt} tensor on the GPU")
    if dets.numel() != amps.numel():
        raise ValueError("dets and amps differ in length")
    with torch.cuda.device(dets.device):  # the library works on the current device
        st = stream if stream is not None else torch.cuda.current_stream(dets.device)
        _chk(lib().swc_energy_noalloc(n_qubits, ctypes.c_void_p(dets.data_ptr()), ctypes.c_void_p(amps.data_ptr()),
                                      dets.numel(), ctypes.c_void_p(h1.data_ptr()), ctypes.c_void_p(h2.data_ptr()),
                                      ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(st.cuda_stream)))


def workspace_bytes(n_qubits, capacity, prec, batch, max_factors, log_capacity=0) -> int:
    return int(lib().swc_workspace_bytes(n_qubits, capacity, prec, batch, max_factors, log_capacity))


class Solver:
    """One context of the library: `batch` sparse states of `n_qubits`
    spin-orbitals in hash tables of `capacity` slots on one GPU."""

    def __init__(self, n_qubits: int, n_alpha: int, n_beta: int, capacity: int, prec: int = FP32,
                 batch: int = 1, max_factors: int = 1, log_capacity: int = 0, device="cuda:0",
                 stream: torch.cuda.Stream | None = None):
        L = lib()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the swc library runs on an MI355X only")
        self.device = torch.device(device)
        self.n_qubits, self.batch, self.prec, self.max_factors = n_qubits, batch, prec, max_factors
        self.capacity = capacity
        nbytes = workspace_bytes(n_qubits, capacity, prec, batch, max_factors, log_capacity)
        if nbytes == 0:
            raise SwcError(EINVAL, "invalid sizes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._ctx = ctypes.c_void_p()
        _chk(L.swc_create(ctypes.byref(self._ctx), n_qubits, n_alpha, n_beta, capacity, prec, batch, max_factors,
                          log_capacity, ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                          ctypes.c_void_p(self.stream.cuda_stream)))
        _open_solvers.add(self)

    # -- helpers ----------------------------------------------------------
    def _dev(self, t, shape=None) -> torch.Tensor:
        t = torch.as_tensor(t, dtype=torch.float64, device=self.device).contiguous()
        if shape is not None and tuple(t.shape) != tuple(shape):
            t = t.reshape(shape).contiguous()
        return t

    def _theta(self, theta, M) -> torch.Tensor:
        t = self._dev(theta)
        if t.dim() == 1:
            t = t.unsqueeze(0).expand(self.batch, M).contiguous()
        if tuple(t.shape) != (self.batch, M):
            raise SwcError(EINVAL, f"theta must be [{self.batch}, {M}]")
        return t

    def _sync_inputs(self):
        # inputs written on torch's current stream must be ready on ours
        if self.stream != torch.cuda.current_stream(self.device):
            self.stream.wait_stream(torch.cuda.current_stream(self.device))

    # -- API ----------------------------------------------------------------
    def build_state(self, dets=None, amps=None):
        if dets is None:
            _chk(lib().swc_build_state(self._ctx, None, None, 0))
            return
        d = np.ascontiguousarray(np.asarray(dets, dtype=np.uint64).reshape(-1))
        a = np.ascontiguousarray(np.asarray(amps, dtype=np.float64).reshape(-1))
        if d.shape != a.shape:
            raise SwcError(EINVAL, "dets and amps differ in length")
        _chk(lib().swc_build_state(self._ctx, _ptr(d), _ptr(a), d.shape[0]))

    def apply_ucc(self, theta, exc, threshold: float = 0.0):
        e = _exc_array(exc)
        M = e.shape[0]
        t = self._theta(theta, M)
        self._sync_inputs()
        _chk(lib().swc_apply_ucc(self._ctx, ctypes.c_void_p(t.data_ptr()), _ptr(e), M, float(threshold)))

    def energy(self, h1, h2) -> torch.Tensor:
        h1d, h2d = self._dev(h1), self._dev(h2)
        E = torch.empty(self.batch, dtype=torch.float64, device=self.device)
        self._sync_inputs()
        _chk(lib().swc_energy(self._ctx, ctypes.c_void_p(h1d.data_ptr()), ctypes.c_void_p(h2d.data_ptr()),
                              ctypes.c_void_p(E.data_ptr())))
        return E

    def energy_and_grad(self, theta, exc, threshold, h1, h2):
        e = _exc_array(exc)
        M = e.shape[0]
        t = self._theta(theta, M)
        h1d, h2d = self._dev(h1), self._dev(h2)
        E = torch.empty(self.batch, dtype=torch.float64, device=self.device)
        g = torch.empty((self.batch, M), dtype=torch.float64, device=self.device)
        self._sync_inputs()
        _chk(lib().swc_energy_and_grad(self._ctx, ctypes.c_void_p(t.data_ptr()), _ptr(e), M, float(threshold),
                                       ctypes.c_void_p(h1d.data_ptr()), ctypes.c_void_p(h2d.data_ptr()),
                                       ctypes.c_void_p(E.data_ptr()), ctypes.c_void_p(g.data_ptr())))
        return E, g

    def set_checkpoints(self, interval: int, max_entries: int = 0):
        """Snapshot the state every `interval` forward steps of a gradient
        sweep (0 turns checkpoints off); `max_entries` live determinants per
        snapshot and batch member (default: the table capacity / 2)."""
        if interval <= 0:
            _chk(lib().swc_set_checkpoints(self._ctx, 0, 0, None, 0))
            self.ckpt_buffer = None
            return
        cap = max_entries if max_entries > 0 else self.capacity // 2
        nbytes = int(lib().swc_checkpoint_bytes(self.prec, self.batch, self.max_factors, interval, cap))
        if nbytes == 0:
            raise SwcError(EINVAL, "invalid checkpoint sizes")
        self.ckpt_buffer = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        _chk(lib().swc_set_checkpoints(self._ctx, interval, cap, ctypes.c_void_p(self.ckpt_buffer.data_ptr()),
                                       nbytes))

    def set_sigma_scratch(self, nbytes: int, mode: int = 0):
        """Device scratch for sigma by pairing two-electron-removed keys
        (mode 0 auto, 1 always, 2 never; nbytes 0 frees it)."""
        if nbytes <= 0:
            _chk(lib().swc_set_sigma_scratch(self._ctx, None, 0, 2))
            self.sigma_buffer = None
            return
        self.sigma_buffer = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        _chk(lib().swc_set_sigma_scratch(self._ctx, ctypes.c_void_p(self.sigma_buffer.data_ptr()), int(nbytes),
                                         int(mode)))

    def set_topk(self, n_max: int, n_cut: int):
        """Keep the n_cut largest |c| after a factor that leaves more than
        n_max determinants (0, 0: off)."""
        _chk(lib().swc_set_topk(self._ctx, int(n_max), int(n_cut)))

    def track_entropy(self, on: bool = True):
        """Record the entropy (Eq. 6) of the state before and after every
        factor of later forward sweeps."""
        _chk(lib().swc_track_entropy(self._ctx, 1 if on else 0))

    def entropy(self, b: int = 0, n: int | None = None) -> np.ndarray:
        """Entropy trajectory [M + 1] of member b from the last forward sweep."""
        n = n if n is not None else self.max_factors + 1
        out = np.full(n, np.nan)
        _chk(lib().swc_get_entropy(self._ctx, b, _ptr(out), n))
        return out[: np.count_nonzero(~np.isnan(out))].copy()

    def track_live(self, on: bool = True):
        """Count the live determinants of every step of later forward sweeps."""
        _chk(lib().swc_track_live(self._ctx, int(bool(on))))

    def live_counts(self, b: int = 0) -> np.ndarray:
        """Live determinants of member b when each step of the last forward
        sweep began, then after its last step: [M + 1] (int64)."""
        out = np.full(self.max_factors + 1, -1, np.int64)
        _chk(lib().swc_get_live_counts(self._ctx, b, _ptr(out), out.shape[0]))
        return out[: np.count_nonzero(out >= 0)].copy()

    def get_state(self, b: int = 0, cap: int | None = None):
        n = ctypes.c_int64(0)
        cap = cap if cap is not None else 1 << 16
        while True:
            d = np.empty(cap, np.uint64)
            a = np.empty(cap, np.float64)
            r = lib().swc_get_state(self._ctx, b, _ptr(d), _ptr(a), cap, ctypes.byref(n))
            if r == ECAPACITY and n.value > cap:
                cap = n.value
                continue
            _chk(r)
            return d[: n.value].copy(), a[: n.value].copy()

    def stats(self) -> dict:
        s = Stats()
        _chk(lib().swc_get_stats(self._ctx, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def close(self):
        """Destroy the context (its graphs, events and capture stream) while
        the HIP runtime is up; the workspace tensor is released with the
        object.  Idempotent."""
        if getattr(self, "_ctx", None) and self._ctx.value:
            # the library's work on its stream must finish before the graphs
            # and events it uses are destroyed
            self.stream.synchronize()
            lib().swc_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()
        _open_solvers.discard(self)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self, _finalizing=sys.is_finalizing):
        # During interpreter shutdown the HIP runtime may already be torn
        # down: make no device call then (the exit hook has closed every
        # context that was still open before finalisation began).  The
        # check is bound at definition: module globals such as `sys` may
        # already be cleared when a solver held by a script's globals dies.
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class UCCEnergy(torch.autograd.Function):
    """E(theta) with the adjoint gradient of the library as backward.

    forward(theta[B, M], solver, exc, threshold, h1, h2) -> E[B]
    """

    @staticmethod
    def forward(ctx, theta, solver: Solver, exc, threshold, h1, h2):
        E, g = solver.energy_and_grad(theta.detach(), exc, threshold, h1, h2)
        ctx.save_for_backward(g)
        ctx.theta_dim = theta.dim()
        return E.to(theta.dtype)

    @staticmethod
    def backward(ctx, gE):
        (g,) = ctx.saved_tensors
        grad = gE.to(g.dtype)[:, None] * g
        if ctx.theta_dim == 1:
            grad = grad.sum(0)
        return grad, None, None, None, None, None


def ucc_energy(theta, solver: Solver, exc, threshold, h1, h2):
    return UCCEnergy.apply(theta, solver, exc, threshold, h1, h2)
