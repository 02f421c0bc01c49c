"""Periodic (infinite-medium) boundaries on the device.

A periodic homogeneous cube is an infinite medium: the constant flux is an
exact eigenvector of the discrete operators at every grid size, so
k = nu_sigma_f / (sigma_t - sigma_s) for one group and
k = nu_sigma_f^T (diag sigma_t - Sigma_s)^{-1} chi for several (the
closed forms of the checker's infinite-medium pins).  This pins the device
path at grid sizes no dense checker can hold, up to 1024^3 nodes with 16
groups and S16.  On small grids every step is also compared with the
checker's dense periodic operator (one sparse LU step from the same iterate).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dense, tt as OT
from paper_2309_03347_amd import workload as W

pytestmark = pytest.mark.gpu


def _unit(v):
    v = v / np.linalg.norm(v)
    return v if v.sum() >= 0 else -v


def _periodic(wl):
    wl.periodic = (True, True, True)
    return wl


@pytest.mark.parametrize("maker", [
    lambda: W.homogeneous(l=3, N=2, seed=31, tol=1e-10),
    lambda: W.inner_box(l=2, G=2, N=4, seed=32, rmax=64, tol=1e-10),
], ids=["homogeneous_n8_S2", "inner_box_n4_G2_S4"])
def test_periodic_steps_match_dense_oracle(cuda, maker):
    from paper_2309_03347_amd.solver import KeffSolver
    wl = _periodic(maker())
    H, S, F = dense.equation_operators(wl)
    lu = spla.splu(H.tocsc())
    s = KeffSolver(wl, rmax=256, kick=8, max_sweeps=60)
    psi = OT.full_vec(s.native.psi().cores())
    k = 1.0
    for step in range(4):
        print(f"periodic {wl.name} step {step}", flush=True)
        rec = s.step()
        ref = lu.solve(S @ psi + (F @ psi) / k)
        kref = k * (F @ ref).sum() / (F @ psi).sum()
        got = OT.full_vec(s.psi_cores())
        assert abs(rec.k - kref) <= 1e-8 * abs(kref), (step, rec.k, kref)
        assert np.linalg.norm(_unit(got) - _unit(ref)) <= 1e-6, step
        psi, k = got, rec.k
    s.close()


def _k_inf(wl):
    st, Ss, nf, chi = wl.sigma_t[0], wl.sigma_s[0], wl.nu_sigma_f[0], wl.chi
    return float(nf @ np.linalg.solve(np.diag(st) - Ss, chi))


@pytest.mark.parametrize("l,G,N", [(5, 1, 4), (7, 4, 8), (10, 16, 16)],
                         ids=["n32_G1_S4", "n128_G4_S8", "n1024_G16_S16"])
def test_periodic_infinite_medium_k_closed_form(cuda, l, G, N):
    from paper_2309_03347_amd.solver import KeffSolver
    wl = _periodic(W.checkerboard(l=l, G=G, N=N, blocks=1, n_mat=1, seed=40 + l, rmax=16,
                                  tol=1e-10, tol_k=1e-12))
    kinf = _k_inf(wl)
    s = KeffSolver(wl)
    ks = []
    for step in range(40):
        rec = s.step()
        ks.append(rec.k)
        print(f"n{wl.n} G{G} S{N} step {step} k {rec.k:.14f} kinf {kinf:.14f} rank {rec.max_rank}",
              flush=True)
        if step > 3 and abs(rec.k - kinf) <= 1e-10 * kinf and rec.dk <= 1e-11:
            break
    assert abs(ks[-1] - kinf) <= 1e-9 * kinf, (ks[-5:], kinf)
    # the converged flux is the constant, a rank-1 train
    assert rec.max_rank <= 2, rec.max_rank
    s.close()


def test_pu239_slab_on_device_tends_to_critical(cuda):
    # The one-dimensional Pu-239 slab of Table tab:1dbench (exactly critical):
    # 256 nodes across 3.707 cm, two nodes with periodic faces in y and z,
    # Gauss-Legendre S4, S8, S16.  The device k equals the checker's dense
    # eigenvalue of the same operator and tends to 1 as the ordinate count grows.
    import json
    import os
    from paper_2309_03347_amd.solver import KeffSolver
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "pu239_slab.json")))
    errs = []
    for N in (4, 8, 16):
        wl = W.slab(N, 8, d["sigma_t"], d["sigma_s"], d["nu"] * d["sigma_f"], d["width_cm"],
                    rmax=32, tol=1e-10, tol_k=1e-12)
        H, S, F = dense.equation_operators(wl)
        k_ref = dense.k_dominant(H, S, F)
        s = KeffSolver(wl)
        s.run(max_steps=200, tol_k=1e-12)
        print(f"slab S{N}: device k {s.k:.12f} checker {k_ref:.12f} steps {len(s.history)}",
              flush=True)
        assert abs(s.k - k_ref) <= 1e-8 * k_ref
        errs.append(abs(1.0 - s.k))
        s.close()
    assert errs[0] > errs[1] > errs[2]
