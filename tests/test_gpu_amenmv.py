"""Approximate TT matrix-vector product by alternating sweeps (tt_amen_mv).

The product A x is projected core by core onto the current orthonormal
interfaces of y, enriched with the residual and rounded (the amen_mv route of
Section 3.3, eq. mv_obj).  Checked against the checker's dense A x: with the
tolerance governing, y equals A x to the tolerance, and y's ranks stay at the
numerical ranks of A x's unfoldings instead of the R_k r_k of the exact
product.
"""
import numpy as np
import pytest

from oracle import tt as OT

pytestmark = pytest.mark.gpu


def _rand_tt(rng, modes, ranks):
    r = [1] + list(ranks) + [1]
    return [rng.standard_normal((r[k], modes[k], r[k + 1])) for k in range(len(modes))]


def _rand_ttm(rng, modes, ranks):
    R = [1] + list(ranks) + [1]
    return [rng.standard_normal((R[k], modes[k], modes[k], R[k + 1])) for k in range(len(modes))]


@pytest.mark.parametrize("modes,Rk,rk", [
    ((2,) * 8, (2, 3, 3, 3, 3, 3, 2), (2, 3, 4, 4, 4, 3, 2)),
    ((4, 3, 2, 2, 5), (3, 4, 2, 2), (2, 3, 3, 2)),
    ((8,) + (2,) * 7, (3, 4, 4, 3, 3, 2, 2), (4, 5, 5, 4, 3, 2, 2)),
])
def test_amen_mv_matches_dense_product(cuda, modes, Rk, rk):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(sum(modes))
    A = _rand_ttm(rng, modes, Rk)
    x = _rand_tt(rng, modes, rk)
    ref = OT.matvec(A, x)
    cap = [1] + [a * b for a, b in zip(Rk, rk)] + [1]
    dA, dx = native.DeviceTTMat(A), native.DeviceTT.from_cores(x)
    dy = native.DeviceTT(modes, cap)
    info = native.tt_amen_mv(dA, dx, dy, tol=1e-12, rmax=1000, max_sweeps=30)
    y = OT.full_vec(dy.cores())
    print(f"amen_mv {modes}: sweeps {info['sweeps']} ranks {list(dy.r)} "
          f"err {np.linalg.norm(y - ref) / np.linalg.norm(ref):.2e}", flush=True)
    assert np.linalg.norm(y - ref) <= 1e-9 * np.linalg.norm(ref)
    for k in range(1, len(modes)):
        s = OT.unfolding_svals(ref, modes, k)
        assert dy.r[k] <= np.sum(s > 1e-13 * s[0]) + 1, (k, dy.r[k])
    assert max(dy.r) <= max(cap)


def test_amen_mv_rank_cap(cuda):
    # with the rank cap binding, the product is a rank-capped approximation
    # whose error is at least the optimal truncation of the middle unfolding
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(9)
    modes = (2,) * 8
    A = _rand_ttm(rng, modes, (2, 3, 3, 3, 3, 3, 2))
    x = _rand_tt(rng, modes, (2, 3, 4, 4, 4, 3, 2))
    ref = OT.matvec(A, x)
    dy = native.DeviceTT(modes, [1] + [6] * 7 + [1])
    native.tt_amen_mv(native.DeviceTTMat(A), native.DeviceTT.from_cores(x), dy, tol=1e-12,
                      rmax=4, max_sweeps=10)
    assert max(dy.r) <= 4
    s = OT.unfolding_svals(ref, modes, 4)
    y = OT.full_vec(dy.cores())
    assert np.linalg.norm(y - ref) >= np.sqrt((s[4:] ** 2).sum()) * (1 - 1e-9)
    assert np.linalg.norm(y - ref) <= 0.5 * np.linalg.norm(ref)
