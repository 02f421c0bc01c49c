"""Device kernels behind the C ABI against the dense checker (FP64)."""
import numpy as np
import pytest

from oracle import tt as OT

pytestmark = pytest.mark.gpu


def _rand_tt(rng, modes, ranks):
    r = [1] + list(ranks) + [1]
    return [rng.standard_normal((r[k], modes[k], r[k + 1])) for k in range(len(modes))]


def _rand_ttm(rng, rows, cols, ranks):
    R = [1] + list(ranks) + [1]
    return [rng.standard_normal((R[k], rows[k], cols[k], R[k + 1])) for k in range(len(rows))]


@pytest.mark.parametrize("rows,cols,R,r", [
    ((2, 2, 2), (2, 2, 2), (2, 3), (3, 2)),
    ((4, 3, 2, 2), (3, 3, 2, 2), (3, 5, 2), (2, 4, 3)),
    ((24,) + (2,) * 5, (24,) + (2,) * 5, (7, 9, 5, 3, 2), (5, 8, 8, 4, 2)),
])
def test_matvec_matches_dense(cuda, rows, cols, R, r):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(sum(rows))
    A = _rand_ttm(rng, rows, cols, R)
    x = _rand_tt(rng, cols, r)
    dA = native.DeviceTTMat(A)
    dx = native.DeviceTT.from_cores(x)
    cap = [a * b for a, b in zip([1] + list(R) + [1], [1] + list(r) + [1])]
    dy = native.DeviceTT(rows, cap)
    native.tt_matvec(dA, dx, dy)
    y = dy.cores()
    ref = OT.matvec(A, x)
    assert np.abs(OT.full_vec(y) - ref).max() <= 1e-13 * np.abs(ref).max()
    assert list(dy.r) == cap


def _inflate(rng, x):
    """Same tensor with redundant ranks: x + x - x (exact TT sum, ranks tripled)."""
    from paper_2309_03347_amd import qtt
    neg = [c.copy() for c in x]
    neg[0] = -neg[0]
    return qtt.tt_sum([x, x, neg])


@pytest.mark.parametrize("modes,ranks", [
    ((2,) * 6, (2, 3, 4, 3, 2)),
    ((4, 3, 2, 2, 5), (3, 5, 4, 3)),
    ((8,) + (2,) * 9, (6, 9, 12, 14, 12, 9, 6, 4, 2)),
    # inflated ranks up to 66: SVDs with 4 lanes per Jacobi pair
    ((4,) * 6, (3, 9, 22, 9, 3)),
    # an angle-like core of 80 directions between rank 8 and rank 64 (192
    # inflated): QR of 640 x 192 and SVD of 192 x 128 outside LDS by the
    # global-memory factorizations, QR of 3072 x 24 and SVD of 5120 x 8 by
    # row blocks
    ((8, 80, 16, 8), (8, 64, 8)),
    # rank 140 (420 inflated): SVD of 144 x 144, more than 128 columns
    ((12, 12, 12, 12), (12, 140, 12)),
])
def test_round_recovers_exact_ranks(cuda, modes, ranks):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(len(modes))
    x = _rand_tt(rng, modes, ranks)
    big = _inflate(rng, x)
    d = native.DeviceTT.from_cores(big)
    err = native.tt_round(d, 1e-12, 1000)
    y = d.cores()
    full_x = OT.full_vec(x)
    assert np.linalg.norm(OT.full_vec(y) - full_x) <= 1e-11 * np.linalg.norm(full_x)
    # ranks equal the numerical ranks of the unfoldings
    for k in range(1, len(modes)):
        s = OT.unfolding_svals(full_x, modes, k)
        assert d.r[k] == np.sum(s > 1e-10 * s[0]), (k, d.r[k])
    assert err < 1e-11
    # gauge: cores 1..d-1 right-orthonormal after the right-to-left SVD sweep
    for k in range(1, len(modes)):
        c = y[k].reshape(y[k].shape[0], -1)
        assert np.allclose(c @ c.T, np.eye(c.shape[0]), atol=1e-12)


@pytest.mark.parametrize("modes,ranks,cut,bond", [
    # QR of 5440 x 8 and SVD of 640 x 68 (the shape of the 128^3 S8 angle
    # core's unfolding) by row blocks: three blocks in LDS, their stacked R
    ((72, 80, 8), (68, 8), 40, 1),
    # QR of 640 x 64 and SVD of 5120 x 8 by row blocks
    ((8, 80, 16, 8), (8, 64, 8), 40, 2),
    # SVD of 2304 x 96 by a tree of four block levels (the last stack of
    # 192 rows in LDS), its 96 x 96 R factored in global memory
    ((128, 288, 8), (96, 8), 60, 1),
    # SVD of 768 x 100: three block levels, then the stack of two R factors
    # (200 x 100, beyond LDS) in global memory
    ((128, 96, 8), (100, 8), 60, 1),
])
def test_round_by_row_blocks(cuda, modes, ranks, cut, bond):
    # matrices too tall for LDS are factored in row blocks; the rounding keeps
    # the tensor and its ranks, leaves right-orthonormal cores, and a rank cut
    # on one bond equals the optimal truncation of that bond's unfolding
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(sum(modes))
    x = _rand_tt(rng, modes, ranks)
    full = OT.full_vec(x)
    d = native.DeviceTT.from_cores(x)
    native.tt_round(d, 1e-13, 1000)
    y = d.cores()
    assert list(d.r[1:-1]) == list(ranks)
    assert np.linalg.norm(OT.full_vec(y) - full) <= 1e-12 * np.linalg.norm(full)
    for k in range(1, len(modes)):
        c = y[k].reshape(y[k].shape[0], -1)
        assert np.allclose(c @ c.T, np.eye(c.shape[0]), atol=1e-12), k
    d2 = native.DeviceTT.from_cores(x)
    native.tt_round(d2, 1e-14, cut)
    assert d2.r[bond] == cut and max(d2.r) == max(cut, max(r for r in ranks if r <= cut))
    s = OT.unfolding_svals(full, modes, bond)
    best = np.sqrt((s[cut:] ** 2).sum())
    err = np.linalg.norm(OT.full_vec(d2.cores()) - full)
    assert abs(err - best) <= 1e-9 * best, (err, best)


@pytest.mark.parametrize("tol", [1e-2, 1e-4, 1e-6])
def test_round_error_bound(cuda, tol):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(7)
    # decaying spectrum: sum of rank-1 terms with geometric weights
    modes = (2,) * 8
    terms = []
    for t in range(12):
        c = _rand_tt(rng, modes, (1,) * 7)
        c[0] = c[0] * 0.3 ** t
        terms.append(c)
    from paper_2309_03347_amd import qtt
    x = qtt.tt_sum(terms)
    full = OT.full_vec(x)
    d = native.DeviceTT.from_cores(x)
    err = native.tt_round(d, tol, 1000)
    y = OT.full_vec(d.cores())
    true = np.linalg.norm(y - full) / np.linalg.norm(full)
    assert true <= tol * (1 + 1e-8)
    assert abs(true - err) <= 1e-8 + 1e-6 * true
    assert max(d.r) < 12


def test_round_rank_cap_binds(cuda):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(8)
    x = _rand_tt(rng, (2,) * 8, (2, 4, 8, 12, 8, 4, 2))
    d = native.DeviceTT.from_cores(x)
    native.tt_round(d, 1e-14, 3)
    assert max(d.r) == 3
    # the result is the SVD truncation; its error is at least the optimal
    # rank-3 error of the middle unfolding
    full = OT.full_vec(x)
    s = OT.unfolding_svals(full, (2,) * 8, 4)
    best = np.sqrt((s[3:] ** 2).sum())
    y = OT.full_vec(d.cores())
    assert np.linalg.norm(y - full) >= best * (1 - 1e-10)


@pytest.mark.parametrize("modes,ranks", [
    ((8, 80, 16, 8), (8, 64, 8)),     # QR of 5120 x 8 by row blocks
    ((128, 96, 8), (100, 8)),         # QR of 768 x 100 by a tree, global-memory top
])
def test_orth_right_keeps_the_tensor(cuda, modes, ranks):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(12)
    x = _rand_tt(rng, modes, ranks)
    full = OT.full_vec(x)
    d = native.DeviceTT.from_cores(x)
    native.tt_orth_right(d)
    y = d.cores()
    assert np.linalg.norm(OT.full_vec(y) - full) <= 1e-12 * np.linalg.norm(full)
    for k in range(1, len(modes)):
        c = y[k].reshape(y[k].shape[0], -1)
        assert np.allclose(c @ c.T, np.eye(c.shape[0]), atol=1e-12), k


def test_dot_matches_dense(cuda):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(9)
    a = _rand_tt(rng, (3, 2, 2, 4), (2, 3, 2))
    b = _rand_tt(rng, (3, 2, 2, 4), (3, 2, 4))
    v = native.tt_dot(native.DeviceTT.from_cores(a), native.DeviceTT.from_cores(b))
    ref = OT.dot(a, b)
    assert abs(v - ref) <= 1e-13 * max(1.0, abs(ref))


def _local_system(rng, ra, RL, n, RR, rc, shift=8.0):
    import torch
    phiL = rng.standard_normal((ra, RL, ra)) / np.sqrt(ra * RL)
    phiR = rng.standard_normal((rc, RR, rc)) / np.sqrt(rc * RR)
    A = rng.standard_normal((RL, n, n, RR)) / np.sqrt(n)
    # make it well conditioned: add shift * identity through the first rank term
    phiL[:, 0, :] += shift * np.eye(ra)
    phiR[:, 0, :] += np.eye(rc)
    A[0, :, :, 0] += np.eye(n)
    if n > 2:
        # angle-like core: diagonal in the mode, as the transport operator is
        A = np.einsum("bijc,ij->bijc", A, np.eye(n))
    f = rng.standard_normal(ra * n * rc)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return phiL, A, phiR, f, t


@pytest.mark.parametrize("method,ra,RL,n,RR,rc", [
    (1, 3, 2, 2, 3, 4),      # dense solve, N = 24 (register Gauss-Jordan)
    (1, 4, 3, 2, 3, 8),      # N = 64: largest of the smallest register tile
    (1, 5, 3, 2, 3, 13),     # N = 130
    (1, 8, 5, 2, 4, 8),
    (1, 7, 3, 2, 3, 10),     # N = 140
    (1, 9, 3, 2, 3, 8),      # N = 144: largest of its register tile
    (1, 6, 3, 2, 3, 16),     # N = 192: largest all-register solve
    (1, 7, 3, 2, 3, 14),     # N = 196: two column blocks in LDS
    (1, 9, 3, 2, 3, 13),     # N = 234, a system of the 32^3 case
    (1, 8, 3, 2, 3, 15),     # N = 240: largest Gauss-Jordan solve
    (1, 5, 3, 2, 4, 25),     # N = 250: blocked LU (panels in LDS)
    (1, 7, 3, 2, 3, 37),     # N = 518: blocked LU, ragged last panel
    (1, 10, 2, 2, 2, 55),    # N = 1100: panel outside LDS, unblocked LU in global memory
    (2, 6, 4, 2, 5, 7),      # GMRES
    (2, 16, 6, 2, 6, 16),
    (0, 4, 3, 24, 3, 5),     # automatic (angle-like core): 24 blocks of 20
    (3, 4, 3, 3, 3, 36),     # blocks of 144, as at the angle core of the 32^3 case
    (3, 6, 3, 3, 3, 32),     # blocks of 192
    (3, 5, 3, 3, 3, 40),     # blocks of 200: blocked LU
    (3, 8, 3, 6, 3, 68),     # blocks of 544 (rank 8 | rank 64 + kick): blocked LU
    (3, 8, 2, 3, 2, 132),    # blocks of 1056: the largest blocked-LU panel
])
def test_local_solve_matches_dense(cuda, method, ra, RL, n, RR, rc):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(ra * 100 + rc)
    phiL, A, phiR, f, t = _local_system(rng, ra, RL, n, RR, rc)
    M = OT.local_matrix(phiL, A, phiR)
    ref = np.linalg.solve(M, f)
    x0 = np.zeros_like(f)
    x, info = native.tt_local_solve(t(phiL), t(A), t(phiR), t(f.reshape(ra, n, rc)),
                                    t(x0.reshape(ra, n, rc)), method=method, tol=1e-12,
                                    max_iter=3000, restart=120, direct_max=128)
    x = x.cpu().numpy().reshape(-1)
    cond = np.linalg.cond(M)
    assert info["converged"], (info, cond)
    assert np.linalg.norm(x - ref) <= 1e-12 * cond * np.linalg.norm(ref), (info, cond)
    assert info["rel_res"] <= 1e-11, info
