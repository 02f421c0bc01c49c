"""Thin ctypes binding of libttnt.so (include/ttnt.h).

Argument marshalling only: every numerical step runs in the HIP library.
PyTorch supplies device memory and the current stream.  Importing this
module never falls back to anything: if the compiled library is missing,
``lib()`` raises ``NativeLibraryMissing``.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttnt.so")

TT_OK, TT_E_ARG, TT_E_CAPACITY, TT_E_NOCONV, TT_E_NUMERIC, TT_E_DTYPE, TT_E_HIP = 0, -1, -2, -3, -4, -5, -6
_NAMES = {0: "TT_OK", -1: "TT_E_ARG", -2: "TT_E_CAPACITY", -3: "TT_E_NOCONV",
          -4: "TT_E_NUMERIC", -5: "TT_E_DTYPE", -6: "TT_E_HIP"}

EXPORTED = ["ttnt_version", "tt_last_error", "tt_matvec", "tt_round_workspace", "tt_round",
            "tt_dot_workspace", "tt_dot", "tt_local_solve_workspace", "tt_local_solve",
            "tt_solver_create", "tt_power_step", "tt_solver_get_psi", "tt_solver_ranks",
            "tt_solver_launches", "tt_solver_destroy", "tt_solver_set_probe",
            "tt_solver_probe_stats", "tt_power_step_batched", "tt_local_solve_noalloc",
            "ttnt_set_grid_wait_limit", "tt_orth_right", "tt_local_apply_workspace",
            "tt_local_apply", "ttnt_release", "tt_amen_mv", "tt_solver_workspace_size",
            "tt_solver_create_in", "tt_power_step_async", "ttnt_set_grid_cap"]


class NativeLibraryMissing(RuntimeError):
    pass


class TTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


I32P = ctypes.POINTER(ctypes.c_int32)
I64P = ctypes.POINTER(ctypes.c_int64)


class TTVec(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n", I32P), ("r", I32P), ("rcap", I32P),
                ("data", ctypes.c_void_p), ("off", I64P)]


class TTMat(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("m", I32P), ("n", I32P), ("R", I32P),
                ("data", ctypes.c_void_p), ("off", I64P)]


class TTLocal(ctypes.Structure):
    _fields_ = [("ra", ctypes.c_int32), ("RL", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n", ctypes.c_int32), ("RR", ctypes.c_int32), ("rc", ctypes.c_int32),
                ("phiL", ctypes.c_void_p), ("A", ctypes.c_void_p), ("phiR", ctypes.c_void_p),
                ("f", ctypes.c_void_p)]


class TTSolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("direct_max", ctypes.c_int32), ("precision", ctypes.c_int32)]


class TTSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("method_used", ctypes.c_int32),
                ("rel_res", ctypes.c_double)]


class TTProblem(ctypes.Structure):
    _fields_ = [("H", TTMat), ("SF", TTMat), ("F_core0", ctypes.c_void_p), ("cF", TTVec),
                ("psi0", TTVec), ("k0", ctypes.c_double)]


class TTSolverOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("rmax", ctypes.c_int32), ("kick", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("rhs_mode", ctypes.c_int32),
                ("rhs_rmax", ctypes.c_int32), ("local_tol", ctypes.c_double),
                ("gmres_restart", ctypes.c_int32), ("gmres_max_iter", ctypes.c_int32),
                ("direct_max", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("min_sweeps", ctypes.c_int32), ("cap_eta", ctypes.c_double),
                ("stall", ctypes.c_double), ("krylov_path", ctypes.c_int32)]


class TTProbeStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("dropped", ctypes.c_int64)]


PROBE_CLASSES = {0: "gemm_nn", 1: "gemm_tn", 2: "gemm_nt", 3: "gemm_tt", 4: "arnoldi",
                 5: "core_matvec", 6: "krylov", 7: "gemm_bf16"}


class TTStepInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_double), ("k_prev", ctypes.c_double), ("dk", ctypes.c_double),
                ("max_local_res", ctypes.c_double), ("trunc_err", ctypes.c_double),
                ("sweeps", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("local_iters", ctypes.c_int32), ("status", ctypes.c_int32)]


_lib = None


def lib():
    """Load libttnt.so (built in-tree); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NativeLibraryMissing(
                f"{LIB_PATH} not found: build it with paper_2309_03347_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        v = ctypes.c_void_p
        L.ttnt_version.restype = ctypes.c_int32
        L.tt_last_error.restype = ctypes.c_char_p
        L.tt_matvec.argtypes = [ctypes.POINTER(TTMat), ctypes.POINTER(TTVec),
                                ctypes.POINTER(TTVec), v]
        L.tt_round_workspace.argtypes = [ctypes.POINTER(TTVec)]
        L.tt_round_workspace.restype = ctypes.c_size_t
        L.tt_round.argtypes = [ctypes.POINTER(TTVec), ctypes.c_double, ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_double), v, ctypes.c_size_t, v]
        L.tt_dot_workspace.argtypes = [ctypes.POINTER(TTVec), ctypes.POINTER(TTVec)]
        L.tt_dot_workspace.restype = ctypes.c_size_t
        L.tt_dot.argtypes = [ctypes.POINTER(TTVec), ctypes.POINTER(TTVec),
                             ctypes.POINTER(ctypes.c_double), v, ctypes.c_size_t, v]
        L.tt_local_solve_workspace.argtypes = [ctypes.POINTER(TTLocal), ctypes.POINTER(TTSolveOpts)]
        L.tt_local_solve_workspace.restype = ctypes.c_size_t
        L.tt_local_solve.argtypes = [ctypes.POINTER(TTLocal), v, ctypes.POINTER(TTSolveOpts),
                                     ctypes.POINTER(TTSolveInfo), v, ctypes.c_size_t, v]
        L.tt_local_solve_noalloc.argtypes = [ctypes.POINTER(TTLocal), v,
                                             ctypes.POINTER(TTSolveOpts),
                                             ctypes.POINTER(TTSolveInfo), v]
        L.ttnt_set_grid_wait_limit.argtypes = [ctypes.c_double]
        L.tt_orth_right.argtypes = [ctypes.POINTER(TTVec), v, ctypes.c_size_t, v]
        L.ttnt_release.argtypes = []
        L.tt_amen_mv.argtypes = [ctypes.POINTER(TTMat), ctypes.POINTER(TTVec), ctypes.POINTER(TTVec),
                                 ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(TTStepInfo), v]
        L.tt_local_apply_workspace.argtypes = [ctypes.POINTER(TTLocal)]
        L.tt_local_apply_workspace.restype = ctypes.c_size_t
        L.tt_local_apply.argtypes = [ctypes.POINTER(TTLocal), v, v, ctypes.c_int32, v,
                                     ctypes.c_size_t, v]
        L.tt_solver_create.argtypes = [ctypes.POINTER(TTProblem), ctypes.POINTER(TTSolverOpts),
                                       ctypes.POINTER(v)]
        L.tt_solver_workspace_size.argtypes = [ctypes.POINTER(TTProblem),
                                               ctypes.POINTER(TTSolverOpts),
                                               ctypes.POINTER(ctypes.c_size_t)]
        L.tt_solver_create_in.argtypes = [ctypes.POINTER(TTProblem), ctypes.POINTER(TTSolverOpts),
                                          v, ctypes.c_size_t, ctypes.POINTER(v)]
        L.tt_power_step.argtypes = [v, ctypes.POINTER(TTStepInfo), v]
        L.tt_power_step_async.argtypes = [v, ctypes.c_int32, v, v]
        L.ttnt_set_grid_cap.argtypes = [ctypes.c_int32]
        L.tt_power_step_batched.argtypes = [ctypes.POINTER(v), ctypes.c_int32,
                                            ctypes.POINTER(TTStepInfo), ctypes.POINTER(v),
                                            ctypes.c_int32]
        L.tt_solver_get_psi.argtypes = [v, ctypes.POINTER(TTVec), v]
        L.tt_solver_ranks.argtypes = [v, I32P, I32P]
        L.tt_solver_launches.argtypes = [v]
        L.tt_solver_launches.restype = ctypes.c_int64
        L.tt_solver_destroy.argtypes = [v]
        L.tt_solver_set_probe.argtypes = [v, ctypes.c_int32]
        L.tt_solver_probe_stats.argtypes = [v, ctypes.c_int32, ctypes.POINTER(TTProbeStats)]
        for name in EXPORTED:
            if name not in ("ttnt_version", "tt_last_error", "tt_round_workspace",
                            "tt_dot_workspace", "tt_local_solve_workspace",
                            "tt_solver_launches", "tt_local_apply_workspace"):
                getattr(L, name).restype = ctypes.c_int32
        _lib = L
    return _lib


def set_grid_cap(cap: int) -> None:
    """Cap the persistent GMRES grids this thread launches (0: default)."""
    _check(lib().ttnt_set_grid_cap(int(cap)))


def step_info_buffer():
    """A device buffer for tt_power_step_async's tt_step_info."""
    torch = _torch()
    return torch.zeros(ctypes.sizeof(TTStepInfo), dtype=torch.uint8, device="cuda")


def read_step_info(buf) -> dict:
    """Decode a device tt_step_info (copies it to the host; synchronizes)."""
    raw = bytes(buf.cpu().numpy().tobytes())
    return _info_dict(TTStepInfo.from_buffer_copy(raw))


def _check(status: int, allow=()):
    if status != TT_OK and status not in allow:
        msg = lib().tt_last_error()
        raise TTError(status, msg.decode() if msg else "")
    return status


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _i32(a):
    arr = np.ascontiguousarray(a, dtype=np.int32)
    return arr, arr.ctypes.data_as(I32P)


def _i64(a):
    arr = np.ascontiguousarray(a, dtype=np.int64)
    return arr, arr.ctypes.data_as(I64P)


class DeviceTT:
    """TT vector in one device buffer with per-core capacity slots."""

    def __init__(self, n: Sequence[int], rcap: Sequence[int], device="cuda"):
        torch = _torch()
        self.d = len(n)
        self.n = np.array(n, dtype=np.int32)
        self.rcap = np.array(rcap, dtype=np.int32)
        self.r = np.ones(self.d + 1, dtype=np.int32)
        sizes = [int(self.rcap[k]) * int(self.n[k]) * int(self.rcap[k + 1]) for k in range(self.d)]
        self.off = np.zeros(self.d, dtype=np.int64)
        self.off[1:] = np.cumsum(sizes)[:-1]
        self.buf = torch.zeros(max(1, int(sum(sizes))), dtype=torch.float64, device=device)

    @classmethod
    def from_cores(cls, cores, rcap=None, device="cuda"):
        torch = _torch()
        n = [c.shape[1] for c in cores]
        r = [cores[0].shape[0]] + [c.shape[-1] for c in cores]
        rcap = r if rcap is None else [max(a, b) for a, b in zip(rcap, r)]
        t = cls(n, rcap, device)
        t.r[:] = r
        for k, c in enumerate(cores):
            flat = torch.from_numpy(np.ascontiguousarray(c, dtype=np.float64).reshape(-1))
            t.buf[int(t.off[k]):int(t.off[k]) + flat.numel()].copy_(flat)
        return t

    def cores(self) -> List[np.ndarray]:
        host = self.buf.detach().cpu().numpy()
        out = []
        for k in range(self.d):
            sz = int(self.r[k]) * int(self.n[k]) * int(self.r[k + 1])
            o = int(self.off[k])
            out.append(host[o:o + sz].reshape(int(self.r[k]), int(self.n[k]), int(self.r[k + 1])).copy())
        return out

    def desc(self) -> TTVec:
        self._keep = (self.n, self.rcap, self.off)
        return TTVec(self.d, self.n.ctypes.data_as(I32P), self.r.ctypes.data_as(I32P),
                     self.rcap.ctypes.data_as(I32P), ctypes.c_void_p(self.buf.data_ptr()),
                     self.off.ctypes.data_as(I64P))


class DeviceTTMat:
    """TT matrix, cores packed contiguously on the device."""

    def __init__(self, cores, device="cuda"):
        torch = _torch()
        self.d = len(cores)
        self.m = np.array([c.shape[1] for c in cores], dtype=np.int32)
        self.n = np.array([c.shape[2] for c in cores], dtype=np.int32)
        self.R = np.array([cores[0].shape[0]] + [c.shape[-1] for c in cores], dtype=np.int32)
        sizes = [c.size for c in cores]
        self.off = np.zeros(self.d, dtype=np.int64)
        self.off[1:] = np.cumsum(sizes)[:-1]
        flat = np.concatenate([np.ascontiguousarray(c, dtype=np.float64).reshape(-1) for c in cores])
        self.buf = torch.from_numpy(flat).to(device)

    def desc(self) -> TTMat:
        return TTMat(self.d, self.m.ctypes.data_as(I32P), self.n.ctypes.data_as(I32P),
                     self.R.ctypes.data_as(I32P), ctypes.c_void_p(self.buf.data_ptr()),
                     self.off.ctypes.data_as(I64P))


def _workspace(nbytes: int):
    torch = _torch()
    return torch.empty(max(1, (int(nbytes) + 7) // 8), dtype=torch.float64, device="cuda")


def tt_matvec(A: DeviceTTMat, x: DeviceTT, y: DeviceTT) -> DeviceTT:
    """y = A x (exact core contraction); y must have capacity R_k r_k."""
    yd = y.desc()
    _check(lib().tt_matvec(ctypes.byref(A.desc()), ctypes.byref(x.desc()), ctypes.byref(yd),
                           _stream()))
    return y


def tt_round(x: DeviceTT, tol: float, rmax: int) -> float:
    """In-place TT rounding; returns the relative discarded norm."""
    xd = x.desc()
    nbytes = lib().tt_round_workspace(ctypes.byref(xd))
    ws = _workspace(nbytes)
    err = ctypes.c_double(0.0)
    _check(lib().tt_round(ctypes.byref(xd), float(tol), int(rmax), ctypes.byref(err),
                          ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * 8),
                          _stream()))
    return err.value


def tt_orth_right(x: DeviceTT) -> None:
    """In-place right orthogonalization of cores 1..d-1 (ranks may shrink)."""
    xd = x.desc()
    nbytes = lib().tt_round_workspace(ctypes.byref(xd))
    ws = _workspace(nbytes)
    _check(lib().tt_orth_right(ctypes.byref(xd), ctypes.c_void_p(ws.data_ptr()),
                               ctypes.c_size_t(ws.numel() * 8), _stream()))


def tt_dot(a: DeviceTT, b: DeviceTT) -> float:
    ad, bd = a.desc(), b.desc()
    nbytes = lib().tt_dot_workspace(ctypes.byref(ad), ctypes.byref(bd))
    ws = _workspace(nbytes)
    out = ctypes.c_double(0.0)
    _check(lib().tt_dot(ctypes.byref(ad), ctypes.byref(bd), ctypes.byref(out),
                        ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * 8), _stream()))
    return out.value


def tt_local_solve(phiL, A, phiR, f, x0, method: int = 0, tol: float = 1e-12,
                   max_iter: int = 1000, restart: int = 80, direct_max: int = 256,
                   precision: int = 0):
    """Solve the projected local system; tensors are float64 CUDA tensors.

    phiL [ra, RL, ra], A [RL, n, n, RR], phiR [rc, RR, rc], f/x0 [ra, n, rc].
    Returns (x, info dict); raises TTError except for TT_E_NOCONV (reported in info).
    """
    torch = _torch()
    ra, RL, _ = phiL.shape
    RL2, m, n, RR = A.shape
    rc = phiR.shape[0]
    tensors = [t.contiguous() for t in (phiL, A, phiR, f)]
    x = x0.contiguous().clone()
    sysd = TTLocal(ra, RL, m, n, RR, rc, *[ctypes.c_void_p(t.data_ptr()) for t in tensors])
    opts = TTSolveOpts(method, tol, max_iter, restart, direct_max, precision)
    nbytes = lib().tt_local_solve_workspace(ctypes.byref(sysd), ctypes.byref(opts))
    ws = _workspace(nbytes)
    info = TTSolveInfo()
    st = lib().tt_local_solve(ctypes.byref(sysd), ctypes.c_void_p(x.data_ptr()), ctypes.byref(opts),
                              ctypes.byref(info), ctypes.c_void_p(ws.data_ptr()),
                              ctypes.c_size_t(ws.numel() * 8), _stream())
    _check(st, allow=(TT_E_NOCONV,))
    torch.cuda.synchronize()
    return x, dict(iterations=info.iterations, method=info.method_used, rel_res=info.rel_res,
                   converged=st == TT_OK)


def tt_local_apply(phiL, A, phiR, x, precision: int = 0):
    """y = (PhiL (x) A (x) PhiR) x; tensors are float64 CUDA tensors.  precision 2:
    BF16 matrix-core contractions, 3: block-scaled FP16 ones (FP32 accumulation)."""
    torch = _torch()
    ra, RL, _ = phiL.shape
    RL2, m, n, RR = A.shape
    rc = phiR.shape[0]
    tensors = [t.contiguous() for t in (phiL, A, phiR)]
    xc = x.contiguous()
    y = torch.empty((ra, m, rc), dtype=torch.float64, device=x.device)
    sysd = TTLocal(ra, RL, m, n, RR, rc, *[ctypes.c_void_p(t.data_ptr()) for t in tensors],
                   ctypes.c_void_p(0))
    ws = _workspace(lib().tt_local_apply_workspace(ctypes.byref(sysd)))
    _check(lib().tt_local_apply(ctypes.byref(sysd), ctypes.c_void_p(xc.data_ptr()),
                                ctypes.c_void_p(y.data_ptr()), int(precision),
                                ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel() * 8),
                                _stream()))
    return y


def tt_local_solve_noalloc(phiL, A, phiR, f, x0, method: int = 0, tol: float = 1e-12,
                           max_iter: int = 1000, restart: int = 80, direct_max: int = 256,
                           precision: int = 0):
    """tt_local_solve on the library's static scratch (no workspace argument)."""
    torch = _torch()
    ra, RL, _ = phiL.shape
    RL2, m, n, RR = A.shape
    rc = phiR.shape[0]
    tensors = [t.contiguous() for t in (phiL, A, phiR, f)]
    x = x0.contiguous().clone()
    sysd = TTLocal(ra, RL, m, n, RR, rc, *[ctypes.c_void_p(t.data_ptr()) for t in tensors])
    opts = TTSolveOpts(method, tol, max_iter, restart, direct_max, precision)
    info = TTSolveInfo()
    st = lib().tt_local_solve_noalloc(ctypes.byref(sysd), ctypes.c_void_p(x.data_ptr()),
                                      ctypes.byref(opts), ctypes.byref(info), _stream())
    _check(st, allow=(TT_E_NOCONV,))
    torch.cuda.synchronize()
    return x, dict(iterations=info.iterations, method=info.method_used, rel_res=info.rel_res,
                   converged=st == TT_OK)


def tt_amen_mv(A: "DeviceTTMat", x: DeviceTT, y: DeviceTT, tol: float, rmax: int,
               max_sweeps: int = 20) -> dict:
    """y ~ A x by alternating sweeps (ranks chosen by tol, capped at rmax)."""
    info = TTStepInfo()
    yd = y.desc()
    st = lib().tt_amen_mv(ctypes.byref(A.desc()), ctypes.byref(x.desc()), ctypes.byref(yd),
                          float(tol), int(rmax), int(max_sweeps), ctypes.byref(info), _stream())
    _check(st, allow=(TT_E_NOCONV,))
    return dict(sweeps=info.sweeps, max_local_res=info.max_local_res, trunc_err=info.trunc_err,
                max_rank=info.max_rank, converged=st == TT_OK)


def release() -> None:
    """Orderly teardown: wait for the device and free the library's per-thread
    event and pinned buffer (destroy every Solver first)."""
    if _lib is not None:
        _check(_lib.ttnt_release())


def set_grid_wait_limit(seconds: float) -> None:
    """Seconds a persistent solve's workgroup waits at a grid barrier (default 20)."""
    _check(lib().ttnt_set_grid_wait_limit(ctypes.c_double(seconds)))


def _info_dict(info) -> dict:
    return dict(k=info.k, k_prev=info.k_prev, dk=info.dk, max_local_res=info.max_local_res,
                trunc_err=info.trunc_err, sweeps=info.sweeps, max_rank=info.max_rank,
                local_iters=info.local_iters, status=info.status)


def power_step_batched(solvers, streams) -> list:
    """One power step of every solver, concurrently on the given torch streams
    (tt_power_step_batched).  Returns the step infos in the solvers' order."""
    torch = _torch()
    n = len(solvers)
    if n == 0:
        return []
    handles = (ctypes.c_void_p * n)(*[s.h.value for s in solvers])
    infos = (TTStepInfo * n)()
    sarr = (ctypes.c_void_p * len(streams))(*[st.cuda_stream for st in streams])
    # the solvers' earlier work was issued on the current stream
    torch.cuda.current_stream().synchronize()
    st = lib().tt_power_step_batched(handles, n, infos, sarr, len(streams))
    _check(st, allow=(TT_E_NOCONV,))
    return [_info_dict(infos[i]) for i in range(n)]


class Solver:
    """Handle of a device power-iteration solver (tt_solver_create ... destroy)."""

    def __init__(self, H: DeviceTTMat, SF: DeviceTTMat, F_core0, cF: DeviceTT, psi0: DeviceTT,
                 k0: float = 1.0, tol: float = 1e-8, rmax: int = 32, kick: int = 4,
                 max_sweeps: int = 20, rhs_mode: int = 0, rhs_rmax: int = 0,
                 local_tol: float = 0.0, gmres_restart: int = 80, gmres_max_iter: int = 2000,
                 direct_max: int = 256, precision: int = 0, min_sweeps: int = 0,
                 cap_eta: float = 0.0, stall: float = 0.0, krylov_path: int = 0,
                 caller_workspace: bool = False):
        """caller_workspace: the device workspace is a torch allocation made
        here (tt_solver_workspace_size, tt_solver_create_in) instead of the
        library's own hipMalloc."""
        self._hold = (H, SF, F_core0, cF, psi0)
        prob = TTProblem(H.desc(), SF.desc(), ctypes.c_void_p(F_core0.data_ptr()), cF.desc(),
                         psi0.desc(), float(k0))
        opts = TTSolverOpts(float(tol), int(rmax), int(kick), int(max_sweeps), int(rhs_mode),
                            int(rhs_rmax), float(local_tol), int(gmres_restart),
                            int(gmres_max_iter), int(direct_max), int(precision),
                            int(min_sweeps), float(cap_eta), float(stall), int(krylov_path))
        h = ctypes.c_void_p()
        self.workspace = None
        if caller_workspace:
            nbytes = ctypes.c_size_t(0)
            _check(lib().tt_solver_workspace_size(ctypes.byref(prob), ctypes.byref(opts),
                                                  ctypes.byref(nbytes)))
            self.workspace = _workspace(nbytes.value)
            _check(lib().tt_solver_create_in(ctypes.byref(prob), ctypes.byref(opts),
                                             ctypes.c_void_p(self.workspace.data_ptr()),
                                             ctypes.c_size_t(self.workspace.numel() * 8),
                                             ctypes.byref(h)))
        else:
            _check(lib().tt_solver_create(ctypes.byref(prob), ctypes.byref(opts),
                                          ctypes.byref(h)))
        self.h = h
        self.d = H.d
        self.n = psi0.n.copy()

    def step(self) -> dict:
        info = TTStepInfo()
        st = lib().tt_power_step(self.h, ctypes.byref(info), _stream())
        _check(st, allow=(TT_E_NOCONV,))
        return _info_dict(info)

    def step_async(self, device_info, sweeps: int = 0) -> None:
        """Enqueue one fixed-rank step with no host synchronization (capturable);
        device_info: a CUDA uint8 tensor of ctypes.sizeof(TTStepInfo) bytes;
        sweeps 0: the solver's max_sweeps."""
        _check(lib().tt_power_step_async(self.h, int(sweeps),
                                         ctypes.c_void_p(device_info.data_ptr()), _stream()))

    def ranks(self) -> np.ndarray:
        r = np.zeros(self.d + 1, dtype=np.int32)
        d = ctypes.c_int32(0)
        _check(lib().tt_solver_ranks(self.h, r.ctypes.data_as(I32P), ctypes.byref(d)))
        return r

    def psi(self) -> DeviceTT:
        r = self.ranks()
        out = DeviceTT(self.n, r)
        od = out.desc()
        _check(lib().tt_solver_get_psi(self.h, ctypes.byref(od), _stream()))
        return out

    def launches(self) -> int:
        return int(lib().tt_solver_launches(self.h))

    def set_probe(self, on: bool):
        _check(lib().tt_solver_set_probe(self.h, 1 if on else 0))

    def probe_stats(self) -> dict:
        out = {}
        for c, name in PROBE_CLASSES.items():
            st = TTProbeStats()
            _check(lib().tt_solver_probe_stats(self.h, c, ctypes.byref(st)))
            out[name] = dict(launches=st.launches, total_ms=st.total_ms, flops=st.flops,
                             bytes=st.bytes, dropped=st.dropped)
        return out

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().tt_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
