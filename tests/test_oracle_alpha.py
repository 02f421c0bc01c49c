"""Pins of the checker's alpha-eigenvalue outer iteration (eq. alpha_eig_fixed_points)."""
import numpy as np
import pytest
import scipy.optimize

from oracle import alpha as OA
from paper_2309_03347_amd import workload as W


def test_alpha_one_group_infinite_medium_closed_form():
    # k(alpha) = nu_sigma_f / (sigma_t + alpha / v - sigma_s) in a reflective
    # homogeneous medium, so k = 1 at alpha = v (nu_sigma_f + sigma_s - sigma_t)
    wl = W.homogeneous(l=2, N=2, seed=31, boundary="reflective")
    st, ss, nf = wl.sigma_t[0, 0], wl.sigma_s[0, 0], wl.nu_sigma_f[0, 0]
    inv_v = np.array([0.5])
    a, hist = OA.alpha_eigenvalue(wl, inv_v)
    assert abs(a - (nf + ss - st) / inv_v[0]) < 1e-9
    assert abs(hist[-1][1] - 1.0) < 1e-9
    # k(alpha) itself at the starting points
    for alpha, k in hist[:2]:
        assert abs(k - nf / (st + alpha * inv_v[0] - ss)) < 1e-9


def test_alpha_multigroup_infinite_medium_root():
    wl = W.checkerboard(l=2, G=3, N=2, blocks=1, n_mat=1, seed=32)
    wl.boundary = "reflective"
    wl.nu_sigma_f = wl.nu_sigma_f * 8.0        # a multiplying medium: k_inf > 1 at alpha = 0
    st, Ss, nf, chi = wl.sigma_t[0], wl.sigma_s[0], wl.nu_sigma_f[0], wl.chi
    inv_v = np.array([0.2, 0.7, 1.5])
    k_inf = lambda al: nf @ np.linalg.solve(np.diag(st + al * inv_v) - Ss, chi)
    assert k_inf(0.0) > 1.0
    root = scipy.optimize.brentq(lambda al: k_inf(al) - 1.0, 0.0, 5.0, xtol=1e-14)
    a, hist = OA.alpha_eigenvalue(wl, inv_v)
    assert abs(a - root) < 1e-8
    assert abs(hist[-1][1] - 1.0) < 1e-9


def test_alpha_term_enters_like_the_total_cross_section():
    # V^{-1} carries the same 8-vertex average as sigma_t: a shift of alpha/v
    # on sigma_t changes nothing else in the workload
    wl = W.inner_box(l=2, G=2, N=2, seed=33)
    inv_v = np.array([0.3, 0.9])
    w2 = OA.shifted(wl, 0.4, inv_v)
    assert np.allclose(w2.sigma_t - wl.sigma_t, 0.4 * inv_v[None, :])
    assert np.array_equal(w2.sigma_s, wl.sigma_s) and np.array_equal(w2.nu_sigma_f, wl.nu_sigma_f)
