"""k- and alpha-eigenvalue iterations on the device (host drivers).

``KeffSolver`` assembles the operators once (host setup, ``operators``),
uploads them, and advances eq. TT_k_eff_fixed_points one step per
``tt_power_step`` call of libttnt.so.  ``AlphaSolver`` runs the outer
alpha iteration of eq. alpha_eig_fixed_points around converged k solves.
"""
from __future__ import annotations

import dataclasses
import time
from typing import List, Optional

import numpy as np

from . import native, operators, qtt


@dataclasses.dataclass
class StepRecord:
    k: float
    dk: float
    sweeps: int
    max_rank: int
    max_local_res: float
    trunc_err: float
    local_iters: int
    seconds: float


def joint_rhs_operator(S, F, tol: float = 1e-13):
    """S and F stacked on a leading selector of core 0, compressed once.

    Returns (cores, F_core0): cores[0] is the S part of core 0, F_core0 the F
    part, and cores[1:] are shared, so that core 0 of S + F/k is
    cores[0] + F_core0 / k.
    """
    S0, F0 = S[0], F[0]
    Rs, Rf = S0.shape[-1], F0.shape[-1]
    m, n = S0.shape[1], S0.shape[2]
    first = np.zeros((1, 2, m, n, Rs + Rf))
    first[0, 0, :, :, :Rs] = S0[0]
    first[0, 1, :, :, Rs:] = F0[0]
    rest = []
    if len(S) > 1:
        # block-diagonal chain of the remaining cores (S block first)
        for k in range(1, len(S)):
            a, b = S[k], F[k]
            last = k == len(S) - 1
            core = np.zeros((a.shape[0] + b.shape[0],) + a.shape[1:3] +
                            ((1,) if last else (a.shape[-1] + b.shape[-1],)))
            if last:
                core[:a.shape[0], :, :, 0] = a[:, :, :, 0]
                core[a.shape[0]:, :, :, 0] = b[:, :, :, 0]
            else:
                core[:a.shape[0], :, :, :a.shape[-1]] = a
                core[a.shape[0]:, :, :, a.shape[-1]:] = b
            rest.append(core)
    cores = [first.reshape(1, 2 * m, n, Rs + Rf)] + rest
    if len(cores) > 1:
        cores = qtt.tt_round_host(cores, tol)
    c0 = cores[0].reshape(1, 2, m, n, -1)
    return [c0[:, 0].copy()] + cores[1:], c0[:, 1].copy()


class KeffSolver:
    def __init__(self, wl, rmax: Optional[int] = None, tol: Optional[float] = None,
                 kick: int = 4, max_sweeps: int = 20, rhs_mode: int = 0, rhs_rmax: int = 0,
                 direct_max: int = 256, gmres_restart: int = 80, ops=None, precision: int = 0,
                 min_sweeps: int = 0, cap_eta: float = 0.0, stall: float = 0.0,
                 krylov_path: int = 0, caller_workspace: bool = False):
        import torch
        self.wl = wl
        self.rmax = wl.rmax if rmax is None else rmax
        self.tol = wl.tol if tol is None else tol
        t0 = time.perf_counter()
        self.ops = operators.build(wl) if ops is None else ops
        SF, F0 = joint_rhs_operator(self.ops.S, self.ops.F)
        self.SF_cores, self.F0 = SF, F0
        self.setup_seconds = time.perf_counter() - t0
        self.H = native.DeviceTTMat(self.ops.H)
        self.SF = native.DeviceTTMat(SF)
        self.F0_dev = torch.from_numpy(np.ascontiguousarray(F0).reshape(-1)).to("cuda")
        self.cF = native.DeviceTT.from_cores(self.ops.cF)
        self.psi0 = native.DeviceTT.from_cores(self.ops.psi0)
        self.native = native.Solver(self.H, self.SF, self.F0_dev, self.cF, self.psi0, k0=1.0,
                                    tol=self.tol, rmax=self.rmax, kick=kick,
                                    max_sweeps=max_sweeps, rhs_mode=rhs_mode,
                                    rhs_rmax=rhs_rmax, direct_max=direct_max,
                                    gmres_restart=gmres_restart, precision=precision,
                                    min_sweeps=min_sweeps, cap_eta=cap_eta, stall=stall,
                                    krylov_path=krylov_path, caller_workspace=caller_workspace)
        self.history: List[StepRecord] = []

    @property
    def k(self) -> float:
        return self.history[-1].k if self.history else 1.0

    def step(self) -> StepRecord:
        import torch
        t0 = time.perf_counter()
        info = self.native.step()
        torch.cuda.synchronize()
        rec = StepRecord(info["k"], info["dk"], info["sweeps"], info["max_rank"],
                         info["max_local_res"], info["trunc_err"], info["local_iters"],
                         time.perf_counter() - t0)
        self.history.append(rec)
        return rec

    def run(self, max_steps: int = 200, tol_k: Optional[float] = None) -> List[StepRecord]:
        tol_k = self.wl.tol_k if tol_k is None else tol_k
        for _ in range(max_steps):
            rec = self.step()
            if rec.dk < tol_k:
                break
        return self.history

    def psi_cores(self):
        return self.native.psi().cores()

    def close(self):
        self.native.close()


def step_batched(solvers: List["KeffSolver"], streams) -> List[StepRecord]:
    """One power step of each KeffSolver, run concurrently on `streams`
    (torch.cuda.Stream objects) by the library's single-threaded scheduler."""
    t0 = time.perf_counter()
    infos = native.power_step_batched([s.native for s in solvers], streams)
    dt = time.perf_counter() - t0
    recs = []
    for s, info in zip(solvers, infos):
        rec = StepRecord(info["k"], info["dk"], info["sweeps"], info["max_rank"],
                         info["max_local_res"], info["trunc_err"], info["local_iters"], dt)
        s.history.append(rec)
        recs.append(rec)
    return recs


class AlphaSolver:
    """Alpha-eigenvalue outer iteration (eq. alpha_eig_fixed_points) on the device.

    The alpha V^{-1} term of eq. OpFormAlphaNTE enters the cell equation
    (eq. Discretized_alphaNTE) with the same 8-vertex average as the total
    cross section, so H(alpha) is the transport operator built with
    sigma_t + alpha / v_g.  Each outer step runs the k power iteration of
    H(alpha) psi = (S + F / k) psi to convergence with tt_power_step (the
    previous alpha's flux as the start); alpha starts at 0 and 0.01 and is
    updated by the secant step on k(alpha) = 1.
    """

    def __init__(self, wl, inv_v, alpha0: float = 0.0, alpha1: float = 0.01, **solver_kw):
        self.wl = wl
        self.inv_v = np.asarray(inv_v, dtype=np.float64)
        assert self.inv_v.shape == (wl.G,)
        self.alpha0, self.alpha1 = float(alpha0), float(alpha1)
        self.solver_kw = solver_kw
        self.history: List[tuple] = []     # (alpha, k, power steps)

    def k_of_alpha(self, alpha: float, max_steps: int, tol_k: float, psi0=None) -> tuple:
        w = dataclasses.replace(self.wl, sigma_t=self.wl.sigma_t + alpha * self.inv_v[None, :])
        ops = operators.build(w)
        if psi0 is not None:
            ops.psi0 = psi0
        s = KeffSolver(w, ops=ops, **self.solver_kw)
        s.run(max_steps=max_steps, tol_k=tol_k)
        rec = (alpha, s.k, len(s.history))
        psi = [c.copy() for c in s.psi_cores()]
        s.close()
        return rec, psi

    def run(self, tol_alpha: float = 1e-8, tol_k: float = 1e-10, max_outer: int = 30,
            max_steps: int = 400) -> float:
        r0, psi = self.k_of_alpha(self.alpha0, max_steps, tol_k)
        r1, psi = self.k_of_alpha(self.alpha1, max_steps, tol_k, psi)
        self.history = [r0, r1]
        (a_prev, k_prev, _), (a, k, _) = r0, r1
        for _ in range(max_outer):
            if k == k_prev:
                break
            a_next = a + (1.0 - k) * (a - a_prev) / (k - k_prev)
            rec, psi = self.k_of_alpha(a_next, max_steps, tol_k, psi)
            self.history.append(rec)
            done = abs(a_next - a) <= tol_alpha * max(1.0, abs(a_next))
            a_prev, k_prev, a, k = a, k, a_next, rec[1]
            if done:
                break
        return a
