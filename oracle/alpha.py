"""Alpha-eigenvalue outer iteration on the checker (eq. alpha_eig_fixed_points).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The alpha problem (eq. OpFormAlphaNTE) adds alpha V^{-1} to H.  In the cell
equation (eq. Discretized_alphaNTE) that term is (alpha / v_g) times the
8-vertex average, exactly like the total cross section, so H(alpha) is H
with sigma_t[m, g] replaced by sigma_t[m, g] + alpha / v_g.  Each outer step
solves the k-eigenproblem of H(alpha) to convergence with the exact sweep
iteration; alpha starts at 0 and 0.01 and is updated so that k(alpha) = 1.
The printed update is read as the secant step on k(alpha) - 1:
    alpha+ = alpha_t + (1 - k_t)(alpha_t - alpha_{t-1}) / (k_t - k_{t-1}).

Pins (tests/test_oracle_alpha.py): in a reflective homogeneous medium
k(alpha) = nu_sigma_f / (sigma_t + alpha / v - sigma_s), so the root is
alpha = v (nu_sigma_f + sigma_s - sigma_t); for several groups the root of
nu_sigma_f^T (diag(sigma_t + alpha / v) - Sigma_s)^{-1} chi = 1 found by a
bracketing root finder.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import sweep


def shifted(wl, alpha: float, inv_v) -> object:
    """The workload with sigma_t[m, g] + alpha / v_g (the alpha V^{-1} term)."""
    inv_v = np.asarray(inv_v, dtype=np.float64)
    return dataclasses.replace(wl, sigma_t=wl.sigma_t + alpha * inv_v[None, :])


def k_of_alpha(wl, alpha: float, inv_v, tol_k: float = 1e-11, max_steps: int = 20000,
               psi0=None):
    """Converged k of H(alpha) psi = (S + F / k) psi by the exact sweep iteration."""
    w = shifted(wl, alpha, inv_v)
    prob = sweep.Problem.from_workload(w)
    start = sweep.dense_psi0(wl) if psi0 is None else psi0
    hist, psi = prob.power_iteration(start, 1.0, tol_k, max_steps)
    return float(hist[-1]), psi


def alpha_eigenvalue(wl, inv_v, alpha0: float = 0.0, alpha1: float = 0.01,
                     tol_alpha: float = 1e-10, tol_k: float = 1e-11, max_outer: int = 60):
    """Returns (alpha, [(alpha_t, k_t), ...]) of the secant outer iteration."""
    k0, psi = k_of_alpha(wl, alpha0, inv_v, tol_k)
    k1, psi = k_of_alpha(wl, alpha1, inv_v, tol_k, psi0=psi)
    hist = [(alpha0, k0), (alpha1, k1)]
    a_prev, k_prev, a, k = alpha0, k0, alpha1, k1
    for _ in range(max_outer):
        if k == k_prev:
            break
        a_next = a + (1.0 - k) * (a - a_prev) / (k - k_prev)
        k_next, psi = k_of_alpha(wl, a_next, inv_v, tol_k, psi0=psi)
        hist.append((a_next, k_next))
        done = abs(a_next - a) <= tol_alpha * max(1.0, abs(a_next))
        a_prev, k_prev, a, k = a, k, a_next, k_next
        if done:
            break
    return a, hist
