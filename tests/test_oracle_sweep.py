"""Pins of the transport-sweep checker against what the discrete problem fixes."""
import json
import os

import numpy as np
import pytest

from oracle import dense, sweep
from paper_2309_03347_amd import workload as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _reflective(wl):
    wl.boundary = "reflective"
    return wl


@pytest.mark.parametrize("l", [2, 3])
def test_infinite_medium_one_group_closed_form(l):
    # Reflective homogeneous cube: the constant flux is an exact discrete
    # eigenvector, so k = nu_sigma_f / (sigma_t - sigma_s).
    wl = _reflective(W.homogeneous(l=l, N=2, seed=11))
    st, ss, nf = wl.sigma_t[0, 0], wl.sigma_s[0, 0], wl.nu_sigma_f[0, 0]
    prob = sweep.Problem.from_workload(wl)
    hist, psi = prob.power_iteration(sweep.dense_psi0(wl), 1.0, 0.0, 3000)
    assert abs(hist[-1] - nf / (st - ss)) < 1e-11 * nf / (st - ss)
    # The cell-averaged scalar flux is flat.  (Vertex values may keep the
    # alternating-sign mode of the vertex scheme: its 8-vertex averages and
    # differences vanish, so it has no source and reflects onto itself.)
    phi8 = prob.phi8(psi)
    assert np.std(phi8) / np.mean(np.abs(phi8)) < 1e-10


def test_infinite_medium_multigroup_closed_form():
    wl = _reflective(W.checkerboard(l=2, G=3, N=2, blocks=1, n_mat=1, seed=13))
    st, Ss, nf, chi = wl.sigma_t[0], wl.sigma_s[0], wl.nu_sigma_f[0], wl.chi
    k_inf = nf @ np.linalg.solve(np.diag(st) - Ss, chi)
    prob = sweep.Problem.from_workload(wl)
    hist, _ = prob.power_iteration(sweep.dense_psi0(wl), 1.0, 1e-14, 20000)
    assert abs(hist[-1] - k_inf) < 1e-10 * k_inf


@pytest.mark.parametrize("maker", [lambda: W.homogeneous(l=2, N=4, seed=3),
                                   lambda: W.inner_box(l=2, G=2, N=2, seed=4)])
def test_sweep_equals_dense_solve(maker):
    wl = maker()
    prob = sweep.Problem.from_workload(wl)
    H, S, F = dense.equation_operators(wl)
    rng = np.random.default_rng(0)
    q = rng.uniform(-1, 1, size=wl.G * wl.M ** 3)
    out = prob.sweep(q)
    # right-hand side rows: q at each cell's row for every direction, 0 on boundary rows
    rhs = np.zeros(prob.n_unknowns)
    idx = dense.cell_row_index(wl)
    C = wl.M ** 3
    t = 0
    for g in range(wl.G):
        for l in range(wl.L):
            rhs[idx[t:t + C]] = q[g * C:(g + 1) * C]
            t += C
    ref = np.linalg.solve(H.toarray(), rhs)
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()


def test_three_assemblies_agree():
    wl = W.inner_box(l=2, G=2, N=4, seed=5)
    H, S, F = dense.equation_operators(wl)
    Ha, Sa, Fa = dense.appendix_cell_rows(wl)
    Ht, St, Ft = dense.tt_form_operators(wl)
    idx = dense.cell_row_index(wl)
    assert abs(H[idx] - Ha).max() < 1e-12
    assert abs(S[idx] - Sa).max() < 1e-14 and abs(F[idx] - Fa).max() < 1e-14
    assert abs(Ht[idx] - H[idx]).max() < 1e-12
    assert abs(St - S).max() < 1e-14 and abs(Ft - F).max() < 1e-14


def test_boundary_equation_count():
    # GL(MK + JM + JK + M + J + K + 1) boundary equations (appendix, after eq. discreteBCs)
    wl = W.homogeneous(l=2, N=2, seed=1)
    G, L, M = wl.G, wl.L, wl.M
    H, S, F = dense.equation_operators(wl)
    expected = G * L * (3 * M * M + 3 * M + 1)
    zero_S = np.sum(np.abs(S).sum(axis=1).A1 == 0)
    zero_F = np.sum(np.abs(F).sum(axis=1).A1 == 0)
    assert zero_S == expected and zero_F == expected
    Ht, St, Ft = dense.tt_form_operators(wl)
    assert np.sum(np.abs(St).sum(axis=1).A1 == 0) == expected


@pytest.mark.parametrize("maker", [lambda: W.homogeneous(l=2, N=2, seed=7),
                                   lambda: W.inner_box(l=2, G=2, N=4, seed=8)])
def test_power_iteration_matches_brute_force(maker):
    wl = maker()
    H, S, F = dense.equation_operators(wl)
    k_ges = dense.k_dominant(H, S, F, dense=True)
    prob = sweep.Problem.from_workload(wl)
    hist, _ = prob.power_iteration(sweep.dense_psi0(wl), 1.0, 1e-14, 5000)
    assert abs(hist[-1] - k_ges) < 1e-10 * k_ges
    # the TT-form arrangement of Section 3.1 has the same eigenvalue
    Ht, St, Ft = dense.tt_form_operators(wl)
    assert abs(dense.k_dominant(Ht, St, Ft, dense=True) - k_ges) < 1e-10 * k_ges


def test_inflow_faces_zero_and_balance():
    wl = W.inner_box(l=3, G=2, N=4, seed=9)
    prob = sweep.Problem.from_workload(wl)
    hist, psi = prob.power_iteration(sweep.dense_psi0(wl), 1.0, 1e-13, 3000)
    k = hist[-1]
    n, M, h = wl.n, wl.M, 1.0 / (wl.n - 1)
    P = psi.reshape(wl.G, wl.L, n, n, n)
    q = wl.quad
    for l in range(wl.L):
        i_in = 0 if q.mu[l] > 0 else n - 1
        j_in = 0 if q.eta[l] > 0 else n - 1
        k_in = 0 if q.xi[l] > 0 else n - 1
        assert np.all(P[:, l, :, :, i_in] == 0) and np.all(P[:, l, :, j_in, :] == 0)
        assert np.all(P[:, l, k_in, :, :] == 0)
    # neutron balance: leakage + absorption = scattering + fission / k, per group,
    # with face leakage from the bilinear face averages of the vertex fluxes.
    mat = wl.cell_material()
    for g in range(wl.G):
        leak = 0.0
        for l in range(wl.L):
            p = P[g, l]
            fx = 0.25 * (p[1:, 1:, :] + p[:-1, 1:, :] + p[1:, :-1, :] + p[:-1, :-1, :])
            fy = 0.25 * (p[1:, :, 1:] + p[:-1, :, 1:] + p[1:, :, :-1] + p[:-1, :, :-1])
            fz = 0.25 * (p[:, 1:, 1:] + p[:, :-1, 1:] + p[:, 1:, :-1] + p[:, :-1, :-1])
            lx = (fx[:, :, -1] - fx[:, :, 0]).sum() * q.mu[l] / h
            ly = (fy[:, -1, :] - fy[:, 0, :]).sum() * q.eta[l] / h
            lz = (fz[-1, :, :] - fz[0, :, :]).sum() * q.xi[l] / h
            leak += q.w[l] * (lx + ly + lz)
        avg = np.zeros((wl.G, M, M, M))
        for gg in range(wl.G):
            for l in range(wl.L):
                p = P[gg, l]
                c8 = sum(p[a:a + M, b:b + M, c:c + M] for a in (0, 1) for b in (0, 1) for c in (0, 1)) / 8
                avg[gg] += q.w[l] * c8
        absorb = (wl.sigma_t[mat, g] * avg[g]).sum()
        src = sum(((wl.sigma_s[mat, g, gp] + wl.chi[g] * wl.nu_sigma_f[mat, gp] / k) * avg[gp]).sum()
                  for gp in range(wl.G))
        assert abs(leak + absorb - src) < 1e-9 * abs(src)


def test_homogeneous_flux_is_mirror_symmetric():
    wl = W.homogeneous(l=3, N=4, seed=10, jitter=0.0)
    prob = sweep.Problem.from_workload(wl)
    hist, psi = prob.power_iteration(sweep.dense_psi0(wl), 1.0, 0.0, 400)
    n = wl.n
    phi = np.einsum("l,glkji->gkji", wl.quad.w, psi.reshape(1, wl.L, n, n, n))[0]
    for ax in range(3):
        assert np.abs(phi - np.flip(phi, axis=ax)).max() < 1e-9 * np.abs(phi).max()
    assert np.abs(phi - phi.transpose(2, 1, 0)).max() < 1e-9 * np.abs(phi).max()


def _slab_problem(N, nx, data):
    """1D slab as a 3D grid with one cell in y and z and reflective y, z faces."""
    mu_gl, w_gl = np.polynomial.legendre.leggauss(N)
    pos = mu_gl > 0
    mu_m, w_m = mu_gl[pos], w_gl[pos] / w_gl[pos].sum()
    per = mu_m.size
    tr = np.sqrt((1 - mu_m ** 2) / 2)
    L = 8 * per
    mu, eta, xi, w = (np.empty(L) for _ in range(4))
    for o in range(8):
        sl = slice(o * per, (o + 1) * per)
        mu[sl] = (1 if o & 1 else -1) * mu_m
        eta[sl] = (1 if o & 2 else -1) * tr
        xi[sl] = (1 if o & 4 else -1) * tr
        w[sl] = w_m / 8
    st = data["sigma_t"]
    return sweep.Problem(1, mu, eta, xi, w, np.zeros(nx - 1, dtype=np.int64), [[st]],
                         [[[data["sigma_s"]]]], [[data["nu"] * data["sigma_f"]]], [1.0],
                         (2, 2, nx), (1.0, 1.0, data["width_cm"] / (nx - 1)),
                         reflective=(True, True, False))


@pytest.mark.slow
def test_pu239_slab_is_critical():
    # Worked example printed in the paper: the bare Pu-239 slab is exactly
    # critical; the discrete k approaches 1 as the ordinate count grows.
    data = json.load(open(os.path.join(HERE, "golden", "pu239_slab.json")))
    errs = []
    for N in (4, 8, 16):
        prob = _slab_problem(N, 257, data)
        hist, _ = prob.power_iteration(np.ones(prob.n_unknowns), 1.0, 1e-12, 20000)
        errs.append(abs(hist[-1] - data["k_eff"]))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-3
