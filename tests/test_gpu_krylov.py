"""Persistent GMRES local solve (method 2, FP64 and mixed) against a dense
solve and against the per-stage launch path (method 4) on the same systems.
The mixed solve runs its Arnoldi cycles in FP32 and refines the FP64
residual, so it is held to the FP64 bar.

The local system is the Galerkin-projected operator of the alternating solve
(Section 3.3): PhiL (x) A_k (x) PhiR acting on a core of shape [ra, n, rc].
The dense reference assembles that matrix with the checker and solves it with
LAPACK.  Shapes span several 64 x 64 tiles with ragged edges, split-K in the
last contraction, and restart lengths that force restarts.
"""
import numpy as np
import pytest

from oracle import tt as OT

pytestmark = pytest.mark.gpu


def _system(rng, ra, RL, n, RR, rc, diag=True, shift=8.0):
    phiL = rng.standard_normal((ra, RL, ra)) / np.sqrt(ra * RL)
    phiR = rng.standard_normal((rc, RR, rc)) / np.sqrt(rc * RR)
    A = rng.standard_normal((RL, n, n, RR)) / np.sqrt(n * RL * RR)
    phiL[:, 0, :] += shift * np.eye(ra)
    phiR[:, 0, :] += np.eye(rc)
    A[0, :, :, 0] += np.eye(n)
    if n > 2 and diag:
        A = np.einsum("bijc,ij->bijc", A, np.eye(n))
    f = rng.standard_normal(ra * n * rc)
    return phiL, A, phiR, f


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


CASES = [
    # ra, RL, n, RR, rc, restart, diag
    (6, 4, 2, 5, 7, 80, True),       # one tile per stage
    (40, 8, 2, 8, 40, 16, True),     # 5 row tiles, 2 output row tiles, restarts
    (20, 6, 2, 6, 70, 40, True),     # ragged column tiles (70 = 64 + 6)
    (9, 5, 3, 4, 11, 12, False),     # general 3-point mode, many restarts
    (16, 6, 2, 6, 16, 88, True),     # longest restart
    (1, 1, 2, 1, 1, 80, True),       # two unknowns
    (36, 6, 2, 8, 36, 80, True),     # rank 32 + enrichment: matrix-core first product, 2592 unknowns
    (32, 4, 2, 6, 32, 80, True),     # rank 32: eight lanes per PhiR row
    (12, 4, 2, 60, 10, 30, True),    # 120 rows of Q_a: every wavefront's second m-tile
    (41, 4, 2, 5, 9, 30, True),      # n r0 = 82 > 80: the general matrix-core form
    (50, 4, 2, 10, 80, 30, True),    # r1 = 80: five n-tiles, ragged k steps of 24
    (30, 5, 3, 50, 20, 40, False),   # n = 3, n RR = 150: four workgroups per slice
    (20, 3, 4, 40, 24, 30, True),    # n = 4, three workgroups per slice
    (24, 4, 2, 40, 23, 30, True),    # three workgroups per slice owning 16, 16 and 14 elements
    (8, 4, 5, 30, 12, 30, False),    # n = 5: the vector-FMA form
    (40, 4, 2, 8, 96, 30, True),     # r1 = 96: six n-tiles, k steps of 20
    (8, 4, 2, 6, 100, 30, True),     # r1 = 100 > 96: the vector-FMA form
]


@pytest.mark.parametrize("ra,RL,n,RR,rc,restart,diag", CASES)
def test_persistent_gmres_matches_dense(cuda, ra, RL, n, RR, rc, restart, diag):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(1000 * ra + 10 * rc + n)
    phiL, A, phiR, f = _system(rng, ra, RL, n, RR, rc, diag)
    M = OT.local_matrix(phiL, A, phiR)
    ref = np.linalg.solve(M, f)
    shape = (ra, n, rc)
    out = {}
    for method, precision in ((2, 0), (4, 0), (2, 1)):
        print(f"local solve method={method} precision={precision} shape={(ra, RL, n, RR, rc)} "
              f"restart={restart}", flush=True)
        x, info = native.tt_local_solve(_t(phiL), _t(A), _t(phiR), _t(f.reshape(shape)),
                                        _t(np.zeros(shape)), method=method, tol=1e-12,
                                        max_iter=2000, restart=restart, direct_max=0,
                                        precision=precision)
        x = x.cpu().numpy().reshape(-1)
        assert info["method"] == method
        assert info["converged"], info
        assert info["rel_res"] <= 1e-11, info
        assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref), info
        out[(method, precision)] = (x, info)
    # same arithmetic up to the order of the reductions
    assert abs(out[(2, 0)][1]["iterations"] - out[(4, 0)][1]["iterations"]) <= 1
    assert np.linalg.norm(out[(2, 0)][0] - out[(4, 0)][0]) <= 1e-10 * np.linalg.norm(ref)


def test_persistent_gmres_zero_rhs_and_exact_guess(cuda):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(3)
    ra, RL, n, RR, rc = 10, 4, 2, 4, 12
    phiL, A, phiR, f = _system(rng, ra, RL, n, RR, rc)
    shape = (ra, n, rc)
    args = (_t(phiL), _t(A), _t(phiR))
    x0 = rng.standard_normal(shape)
    x, info = native.tt_local_solve(*args, _t(np.zeros(shape)), _t(x0), method=2, tol=1e-12)
    assert info["converged"] and info["iterations"] == 0
    assert np.all(x.cpu().numpy() == 0.0)
    ref = np.linalg.solve(OT.local_matrix(phiL, A, phiR), f)
    x, info = native.tt_local_solve(*args, _t(f.reshape(shape)), _t(ref.reshape(shape)),
                                    method=2, tol=1e-10)
    assert info["converged"] and info["iterations"] == 0
    assert np.linalg.norm(x.cpu().numpy().reshape(-1) - ref) <= 1e-14 * np.linalg.norm(ref)


def test_persistent_gmres_iteration_limit(cuda):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(5)
    ra, RL, n, RR, rc = 24, 6, 2, 6, 24
    phiL, A, phiR, f = _system(rng, ra, RL, n, RR, rc)
    shape = (ra, n, rc)
    x, info = native.tt_local_solve(_t(phiL), _t(A), _t(phiR), _t(f.reshape(shape)),
                                    _t(np.zeros(shape)), method=2, tol=1e-14, max_iter=7,
                                    restart=5)
    assert not info["converged"]
    assert info["iterations"] == 7
    M = OT.local_matrix(phiL, A, phiR)
    r = M @ x.cpu().numpy().reshape(-1) - f
    assert np.linalg.norm(r) < 0.9 * np.linalg.norm(f)
    assert abs(info["rel_res"] - np.linalg.norm(r) / np.linalg.norm(f)) <= 1e-10


# Shapes of the 32^3 four-group workload and beyond: R_H r_1 >= 2016, so the
# PhiR stream runs its double-buffered full-block loop.  The explicit local
# matrix would be too large, so the checker applies the operator factored.
LARGE = [
    # ra, RL, n, RR, rc, restart
    (36, 56, 2, 56, 36, 80),     # the bench's rank-36 cores (matrix-core first product)
    (64, 24, 2, 72, 64, 60),     # n r0 = 128: general matrix-core form, 8192 unknowns
    (48, 40, 2, 200, 48, 60),    # operator rank 200: 13 chunks of 16 beta' over four workgroups
]


@pytest.mark.parametrize("ra,RL,n,RR,rc,restart", LARGE)
def test_persistent_gmres_bench_shapes(cuda, ra, RL, n, RR, rc, restart):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(7 * ra + rc)
    phiL, A, phiR, f = _system(rng, ra, RL, n, RR, rc)
    shape = (ra, n, rc)
    out = {}
    for method, precision in ((2, 0), (4, 0), (2, 1)):
        print(f"local solve method={method} precision={precision} shape={(ra, RL, n, RR, rc)}",
              flush=True)
        x, info = native.tt_local_solve(_t(phiL), _t(A), _t(phiR), _t(f.reshape(shape)),
                                        _t(np.zeros(shape)), method=method, tol=1e-12,
                                        max_iter=3000, restart=restart, direct_max=0,
                                        precision=precision)
        x = x.cpu().numpy().reshape(-1)
        assert info["method"] == method and info["converged"], info
        r = OT.local_apply(phiL, A, phiR, x) - f
        assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(f), info
        out[(method, precision)] = x
    assert np.linalg.norm(out[(2, 0)] - out[(4, 0)]) <= 1e-9 * np.linalg.norm(out[(4, 0)])


@pytest.mark.parametrize("ra,RL,n,RR,rc", [
    (36, 6, 2, 8, 36),       # 36 workgroups
    (64, 24, 2, 72, 64),     # 256 workgroups (four per slice)
])
def test_grid_barrier_wait_gives_up_with_an_error(cuda, ra, RL, n, RR, rc):
    # A limit <= 0 makes every workgroup that has to wait give up at once: the
    # solve must end (every workgroup exits) and report TT_E_HIP.  The wait is
    # forced from the host; no workgroup is ever left unable to proceed.
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(11)
    phiL, A, phiR, f = _system(rng, ra, RL, n, RR, rc)
    shape = (ra, n, rc)
    args = (_t(phiL), _t(A), _t(phiR), _t(f.reshape(shape)), _t(np.zeros(shape)))
    native.set_grid_wait_limit(-1.0)
    try:
        with pytest.raises(native.TTError) as e:
            native.tt_local_solve(*args, method=2, tol=1e-12, max_iter=200, restart=40)
        assert e.value.status == native.TT_E_HIP
        assert "gave up" in str(e.value)
    finally:
        native.set_grid_wait_limit(20.0)
    x, info = native.tt_local_solve(*args, method=2, tol=1e-12, max_iter=2000, restart=40)
    assert info["converged"]
    r = OT.local_apply(phiL, A, phiR, x.cpu().numpy().reshape(-1)) - f
    assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(f)
