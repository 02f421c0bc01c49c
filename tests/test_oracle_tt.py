"""Pins of the dense TT reference semantics (oracle/tt.py)."""
import numpy as np
import pytest

from oracle import tt as OT


def _rand_tt(rng, modes, ranks):
    r = [1] + list(ranks) + [1]
    return [rng.standard_normal((r[k], modes[k], r[k + 1])) for k in range(len(modes))]


def test_rank_one_vector_is_kron():
    rng = np.random.default_rng(0)
    vs = [rng.standard_normal(n) for n in (3, 2, 4)]
    cores = [v.reshape(1, -1, 1) for v in vs]
    assert np.allclose(OT.full_vec(cores), np.kron(np.kron(vs[0], vs[1]), vs[2]))


def test_rank_one_matrix_is_kron():
    rng = np.random.default_rng(1)
    ms = [rng.standard_normal((m, n)) for m, n in ((2, 3), (4, 2), (3, 3))]
    cores = [a.reshape(1, *a.shape, 1) for a in ms]
    assert np.allclose(OT.full_mat(cores), np.kron(np.kron(ms[0], ms[1]), ms[2]))


def test_sum_of_kron_terms_matvec():
    rng = np.random.default_rng(2)
    A1 = [rng.standard_normal((2, 2)) for _ in range(3)]
    A2 = [rng.standard_normal((2, 2)) for _ in range(3)]
    # rank-2 TT matrix holding A1[0](x)A1[1](x)A1[2] + A2[0](x)A2[1](x)A2[2]
    c0 = np.stack([A1[0], A2[0]], axis=-1)[None]
    c1 = np.zeros((2, 2, 2, 2))
    c1[0, :, :, 0], c1[1, :, :, 1] = A1[1], A2[1]
    c2 = np.stack([A1[2], A2[2]], axis=0)[..., None]
    dense = np.kron(np.kron(A1[0], A1[1]), A1[2]) + np.kron(np.kron(A2[0], A2[1]), A2[2])
    x = _rand_tt(rng, (2, 2, 2), (2, 2))
    assert np.allclose(OT.matvec([c0, c1, c2], x), dense @ OT.full_vec(x))


def test_qtt_ranks_of_known_functions():
    x = np.linspace(0, 1, 1 << 8)
    assert max(c.shape[-1] for c in OT.qtt_of_function(np.exp(1.7 * x))) == 1
    assert max(c.shape[-1] for c in OT.qtt_of_function(np.sin(5.3 * x))) == 2
    poly = 1 + x - 2 * x ** 2 + 0.5 * x ** 3
    assert max(c.shape[-1] for c in OT.qtt_of_function(poly)) <= 4


def test_unfolding_singular_values_bound_tt_ranks():
    rng = np.random.default_rng(3)
    x = _rand_tt(rng, (3, 4, 5, 2), (2, 3, 2))
    full = OT.full_vec(x)
    for k, r in zip((1, 2, 3), (2, 3, 2)):
        s = OT.unfolding_svals(full, (3, 4, 5, 2), k)
        assert np.sum(s > 1e-12 * s[0]) <= r


def test_local_matrix_single_core_is_the_operator():
    # d = 1: both interfaces are the scalar 1, so the local system is A itself.
    rng = np.random.default_rng(4)
    A = rng.standard_normal((1, 5, 5, 1))
    M = OT.local_matrix(np.ones((1, 1, 1)), A, np.ones((1, 1, 1)))
    assert np.allclose(M, A[0, :, :, 0])


def test_local_matrix_is_projection_of_full_operator():
    # With orthonormal left/right parts, Phi_L (x) A_k (x) Phi_R equals
    # P^T A P where P = X_<k (x) I (x) X_>k^T (the Galerkin projection).
    rng = np.random.default_rng(5)
    modes = (2, 3, 2, 2)
    x = _rand_tt(rng, modes, (2, 3, 2))
    # left-orthonormalize cores 0..k-1, right-orthonormalize k+1..d-1 (k = 2)
    k = 2
    q, r = np.linalg.qr(x[0].reshape(2, 2))
    x[0] = q.reshape(1, 2, 2)
    x[1] = np.einsum("ab,bnc->anc", r, x[1])
    q, r = np.linalg.qr(x[1].reshape(2 * 3, 3))
    x[1] = q.reshape(2, 3, 3)
    x[2] = np.einsum("ab,bnc->anc", r, x[2])
    q, r = np.linalg.qr(x[3].reshape(2, 2).T)
    x[3] = q.T.reshape(2, 2, 1)
    x[2] = np.einsum("anb,cb->anc", x[2], r)
    A = [rng.standard_normal((1 if i == 0 else 2, modes[i], modes[i], 1 if i == 3 else 2))
         for i in range(4)]
    phiL = OT.left_interface(x, A, k)
    phiR = OT.right_interface(x, A, k)
    M = OT.local_matrix(phiL, A[k], phiR)
    XL = OT._partial(x[:k])                  # [6, 3]
    XR = OT._partial_right(x[k + 1:])        # [2, 2]
    P = np.kron(np.kron(XL, np.eye(modes[k])), XR.T)
    full = OT.full_mat(A)
    assert np.allclose(M, P.T @ full @ P, atol=1e-10)
    assert OT.left_orthonormal(x, k)


def test_round_error_helper():
    a = np.ones(10)
    b = a.copy()
    b[0] += 0.1
    assert abs(OT.round_error_bound(a, b) - 0.1 / np.sqrt(10)) < 1e-15


def test_dot_of_rank_one_trains_is_product_of_factor_dots():
    rng = np.random.default_rng(6)
    a = [rng.standard_normal(n) for n in (3, 2, 5)]
    b = [rng.standard_normal(n) for n in (3, 2, 5)]
    ref = np.prod([x @ y for x, y in zip(a, b)])
    got = OT.dot([v.reshape(1, -1, 1) for v in a], [v.reshape(1, -1, 1) for v in b])
    assert abs(got - ref) < 1e-13 * max(1.0, abs(ref))


def test_local_apply_equals_local_matrix():
    rng = np.random.default_rng(7)
    phiL = rng.standard_normal((3, 4, 3))
    A = rng.standard_normal((4, 3, 3, 2))
    phiR = rng.standard_normal((5, 2, 5))
    x = rng.standard_normal(3 * 3 * 5)
    ref = OT.local_matrix(phiL, A, phiR) @ x
    assert np.allclose(OT.local_apply(phiL, A, phiR, x), ref, rtol=1e-13, atol=1e-13)
