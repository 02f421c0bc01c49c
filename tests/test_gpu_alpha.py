"""Alpha-eigenvalue outer iteration on the device (eq. alpha_eig_fixed_points).

Each outer step runs the device k power iteration of H(alpha) psi =
(S + F/k) psi to convergence; alpha follows the secant step on k(alpha) = 1.
The checker runs the same outer iteration around exact sweep iterations.
"""
import numpy as np
import pytest

from oracle import alpha as OA
from paper_2309_03347_amd import workload as W

pytestmark = pytest.mark.gpu


def test_alpha_matches_checker_two_region(cuda):
    from paper_2309_03347_amd.solver import AlphaSolver
    wl = W.inner_box(l=3, G=2, N=2, seed=41, rmax=256, tol=1e-10)
    wl.nu_sigma_f = wl.nu_sigma_f * 16.0          # supercritical: alpha > 0
    inv_v = np.array([0.4, 1.1])
    a_ref, hist_ref = OA.alpha_eigenvalue(wl, inv_v, tol_alpha=1e-11)
    sol = AlphaSolver(wl, inv_v, kick=8, max_sweeps=60)
    a = sol.run(tol_alpha=1e-10, tol_k=1e-11)
    print(f"alpha device {a:.12f} checker {a_ref:.12f} outer {len(sol.history)}", flush=True)
    assert abs(a - a_ref) <= 1e-7 * max(1.0, abs(a_ref))
    assert abs(sol.history[-1][1] - 1.0) <= 1e-8


def test_alpha_periodic_infinite_medium_closed_form(cuda):
    # one group, periodic homogeneous cube: k(alpha) = nu_sigma_f / (sigma_t +
    # alpha / v - sigma_s), root alpha = v (nu_sigma_f + sigma_s - sigma_t)
    from paper_2309_03347_amd.solver import AlphaSolver
    wl = W.homogeneous(l=5, N=4, seed=42, tol=1e-10, rmax=16)
    wl.periodic = (True, True, True)
    st, ss, nf = wl.sigma_t[0, 0], wl.sigma_s[0, 0, 0], wl.nu_sigma_f[0, 0]
    inv_v = np.array([0.5])
    sol = AlphaSolver(wl, inv_v)
    a = sol.run(tol_alpha=1e-10, tol_k=1e-12)
    exact = float((nf + ss - st) / inv_v[0])
    print(f"alpha {a:.12f} closed form {exact:.12f}", flush=True)
    assert abs(a - exact) <= 1e-8
