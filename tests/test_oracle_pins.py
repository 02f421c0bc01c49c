"""Pins of the checker's per-step quantities (not only its converged k).

Every per-step parity verdict compares the checker's k_{t+1} =
k_t sum(F psi_{t+1}) / sum(F psi_t) (eq. k_eff_fixed_points) and its
unnormalized psi_{t+1} = H^{-1} (S + F/k_t) psi_t.  These tests fix the
fission functional, the source and one whole step against the dense
operators assembled independently from the cell equations, and one step of
the reflective infinite medium against its closed form.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dense, sweep
from paper_2309_03347_amd import workload as W


def _cases():
    return [W.inner_box(l=2, G=2, N=4, seed=5),
            W.homogeneous(l=2, N=2, seed=3),
            W.checkerboard(l=2, G=3, N=2, blocks=2, n_mat=3, seed=21)]


def _rand_psi(wl, seed):
    n = wl.n
    rng = np.random.default_rng(seed)
    return rng.uniform(0.1, 1.0, size=wl.G * wl.L * n ** 3)


@pytest.mark.parametrize("wl", _cases(), ids=lambda w: w.name)
def test_fission_total_is_sum_of_F_psi(wl):
    # sum of all entries of F psi (the k update's functional) against the
    # three dense assemblies of F: equation rows, appendix rows, TT form.
    prob = sweep.Problem.from_workload(wl)
    psi = _rand_psi(wl, 1)
    _, _, F = dense.equation_operators(wl)
    _, _, Fa = dense.appendix_cell_rows(wl)
    _, _, Ft = dense.tt_form_operators(wl)
    got = prob.fission_total(psi)
    for Fx in (F, Fa, Ft):
        ref = float((Fx @ psi).sum())
        assert abs(got - ref) <= 1e-13 * abs(ref)


def test_fission_total_sees_material_and_spectrum():
    # A wrong material index or a dropped chi weight must change the sum:
    # the total equals L * sum_c sum_g chi_g * (nu_sigma_f . phi8)[c] / 8 with
    # chi summing to one, so perturbing nu_sigma_f of one material moves it by
    # exactly that material's share.
    wl = W.inner_box(l=2, G=2, N=2, seed=6)
    prob = sweep.Problem.from_workload(wl)
    psi = _rand_psi(wl, 2)
    base = prob.fission_total(psi)
    wl2 = W.inner_box(l=2, G=2, N=2, seed=6)
    wl2.nu_sigma_f = wl2.nu_sigma_f.copy()
    wl2.nu_sigma_f[1, 0] += 1.0
    got = sweep.Problem.from_workload(wl2).fission_total(psi)
    phi8 = prob.phi8(psi).reshape(wl.G, -1)
    in_box = (wl.cell_material().reshape(-1) == 1)
    share = wl.L * 0.125 * phi8[0, in_box].sum()
    assert abs((got - base) - share) <= 1e-12 * abs(share)


@pytest.mark.parametrize("wl", _cases(), ids=lambda w: w.name)
def test_source_is_S_plus_F_over_k_rows(wl):
    # q[g, c] equals the row of (S + F/k) psi at every direction's cell row.
    prob = sweep.Problem.from_workload(wl)
    psi = _rand_psi(wl, 3)
    k = 0.73
    _, S, F = dense.equation_operators(wl)
    rhs = S @ psi + (F @ psi) / k
    q = prob.source(psi, k)
    C = wl.M ** 3
    idx = dense.cell_row_index(wl)
    t = 0
    for g in range(wl.G):
        for _ in range(wl.L):
            assert np.abs(rhs[idx[t:t + C]] - q[g * C:(g + 1) * C]).max() <= 1e-13 * np.abs(q).max()
            t += C


@pytest.mark.parametrize("wl", _cases(), ids=lambda w: w.name)
def test_power_step_equals_dense_step(wl):
    # psi_1 = H^{-1} (S + F/k_0) psi_0 by a sparse LU of the equation-row H,
    # k_1 = k_0 sum(F psi_1) / sum(F psi_0).
    prob = sweep.Problem.from_workload(wl)
    psi0 = _rand_psi(wl, 4)
    k0 = 1.37
    H, S, F = dense.equation_operators(wl)
    psi1 = spla.splu(H.tocsc()).solve(S @ psi0 + (F @ psi0) / k0)
    k1 = k0 * (F @ psi1).sum() / (F @ psi0).sum()
    got, kg = prob.power_step(psi0, k0)
    assert np.abs(got - psi1).max() <= 1e-12 * np.abs(psi1).max()
    assert abs(kg - k1) <= 1e-13 * abs(k1)


def _periodic(wl):
    wl.periodic = (True, True, True)
    return wl


@pytest.mark.parametrize("N", [2, 4])
@pytest.mark.parametrize("k0", [1.0, 0.5, 2.0])
def test_periodic_step_from_constant_flux(N, k0):
    # A periodic homogeneous cube is an infinite medium.  Its operator maps
    # the constant to a constant: differences vanish, the 8-vertex average of
    # a constant is itself and sum_l w_l = 1, so
    # psi_1 = (sigma_s + nu_sigma_f / k_0) / sigma_t and
    # k_1 = k_0 sigma_s/sigma_t + nu_sigma_f/sigma_t.
    wl = _periodic(W.homogeneous(l=2, N=N, seed=11))
    st, ss, nf = wl.sigma_t[0, 0], wl.sigma_s[0, 0], wl.nu_sigma_f[0, 0]
    H, S, F = dense.equation_operators(wl)
    psi0 = np.ones(H.shape[0])
    psi1 = spla.splu(H.tocsc()).solve(S @ psi0 + (F @ psi0) / k0)
    assert np.abs(psi1 - (ss + nf / k0) / st).max() < 1e-12
    k1 = k0 * (F @ psi1).sum() / (F @ psi0).sum()
    assert abs(k1 - (k0 * ss / st + nf / st)) < 1e-13
    # the error to k_inf contracts by exactly sigma_s / sigma_t
    kinf = nf / (st - ss)
    assert abs((k1 - kinf) - (ss / st) * (k0 - kinf)) < 1e-13


def test_periodic_operator_is_nonsingular_and_differs_from_vacuum():
    # Even node counts exclude the vertex scheme's alternating-sign mode
    # (it has no source and vanishing differences) from periodic functions,
    # so H is invertible; mirror rows would leave that mode free.
    wl = _periodic(W.homogeneous(l=2, N=2, seed=11))
    H, _, _ = dense.equation_operators(wl)
    sv = np.linalg.svd(H.toarray(), compute_uv=False)
    assert sv[-1] > 1e-2 * sv[0]
    Hv, _, _ = dense.equation_operators(wl, periodic=(False, False, False))
    assert abs(H - Hv).max() == 1.0


def test_periodic_dense_eigenvalue_is_closed_form():
    wl = _periodic(W.homogeneous(l=2, N=4, seed=12))
    st, ss, nf = wl.sigma_t[0, 0], wl.sigma_s[0, 0], wl.nu_sigma_f[0, 0]
    H, S, F = dense.equation_operators(wl)
    assert abs(dense.k_dominant(H, S, F, dense=True) - nf / (st - ss)) < 1e-11
    wl3 = _periodic(W.checkerboard(l=2, G=3, N=2, blocks=1, n_mat=1, seed=13))
    st3, Ss, nf3, chi = wl3.sigma_t[0], wl3.sigma_s[0], wl3.nu_sigma_f[0], wl3.chi
    k_inf = nf3 @ np.linalg.solve(np.diag(st3) - Ss, chi)
    H3, S3, F3 = dense.equation_operators(wl3)
    assert abs(dense.k_dominant(H3, S3, F3) - k_inf) < 1e-10 * k_inf


def test_periodic_multigroup_step_from_group_constant_flux():
    # Spatially and angularly constant psi_0 with group profile u: psi_1 is
    # constant with profile diag(sigma_t)^{-1} (Sigma_s + chi nu_sigma_f^T / k_0) u.
    wl = _periodic(W.checkerboard(l=2, G=3, N=2, blocks=1, n_mat=1, seed=14))
    st, Ss, nf, chi = wl.sigma_t[0], wl.sigma_s[0], wl.nu_sigma_f[0], wl.chi
    u = np.array([0.7, 1.3, 0.4])
    k0 = 0.9
    H, S, F = dense.equation_operators(wl)
    per = wl.L * wl.n ** 3
    psi0 = np.repeat(u, per)
    psi1 = spla.splu(H.tocsc()).solve(S @ psi0 + (F @ psi0) / k0)
    v = (Ss @ u + chi * (nf @ u) / k0) / st
    assert np.abs(psi1 - np.repeat(v, per)).max() < 1e-12
    k1 = k0 * (F @ psi1).sum() / (F @ psi0).sum()
    assert abs(k1 - k0 * (nf @ v) / (nf @ u)) < 1e-13


def test_lagged_reflective_sweep_and_periodic_operator_share_k():
    # Both are infinite homogeneous media: the sweep checker's lagged mirror
    # faces and the periodic operator converge to the same k.
    wl = W.homogeneous(l=2, N=2, seed=15, boundary="reflective", jitter=0.0)
    hist, _ = sweep.Problem.from_workload(wl).power_iteration(sweep.dense_psi0(wl), 1.0, 0.0, 3000)
    H, S, F = dense.equation_operators(wl, periodic=(True, True, True))
    assert abs(hist[-1] - dense.k_dominant(H, S, F, dense=True)) < 1e-11


def _pu239(N, lx):
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pu239_slab.json")))
    return W.slab(N, lx, d["sigma_t"], d["sigma_s"], d["nu"] * d["sigma_f"], d["width_cm"])


def test_periodic_two_node_slab_equals_reflective_sweep_slab():
    # Two nodes with periodic y and z faces force a y-, z-uniform flux: the
    # one-dimensional slab.  The sweep checker's slab (one cell across y and z,
    # lagged mirror faces) has the same converged k; its lagged faces leave a
    # slowly decaying mode, so the agreement is to 1e-5.
    wl = _pu239(4, 6)
    H, S, F = dense.equation_operators(wl)
    k_dense = dense.k_dominant(H, S, F)
    prob = sweep.Problem.from_workload(wl, reflective=(True, True, False))
    hist, _ = prob.power_iteration(np.ones(prob.n_unknowns), 1.0, 0.0, 4000)
    assert abs(k_dense - hist[-1]) < 1e-5


def test_pu239_slab_periodic_operator_tends_to_critical():
    # Table tab:1dbench: the bare slab is exactly critical; the discrete k of
    # the periodic-face slab approaches 1 as the ordinate count grows
    errs = []
    for N in (4, 8, 16):
        wl = _pu239(N, 8)
        H, S, F = dense.equation_operators(wl)
        errs.append(abs(1.0 - dense.k_dominant(H, S, F)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3
