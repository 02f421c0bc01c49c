"""Dense reference semantics of tensor trains (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions follow Section 2.2 and appendix B:
  * ``full_vec``: X(i_1..i_d) = G_1(i_1) G_2(i_2) ... G_d(i_d)
    (eq. TT-vector), row-major over (i_1, ..., i_d);
  * ``full_mat``: A((i),(j)) = A_1(i_1,j_1) ... A_d(i_d,j_d)
    (eq. TT-matrix-compact), i.e. the Kronecker product for rank 1;
  * ``matvec``: y = A x on the reconstructions; ``dot``: <a, b> on them;
  * ``round_error_bound``: the relative error ||X - Y|| / ||X|| of a rounding,
    from dense reconstructions (the contract is <= tol when the rank cap does
    not bind);
  * ``unfolding_svals``: singular values of the k-th unfolding (library SVD);
  * ``local_matrix``: the projected local operator of the alternating solve,
    Phi_L (x) A_k (x) Phi_R written as an explicit sum of Kronecker products
    over the operator rank indices;
  * ``local_apply``: the same operator applied to a vector without forming it
    (for systems too large for the explicit matrix);
  * ``left_interface``/``right_interface``: the projections of A onto the
    left/right orthonormal parts of X, computed on the reconstructions of the
    partial trains (no core-wise recursion).

Pins (tests/test_oracle_tt.py): rank-1 reconstructions equal numpy.kron;
QTT of exp(a x) has rank 1 and of sin(a x) rank 2; a matvec of Kronecker
operators equals the Kronecker product applied to a dense vector; the local
matrix of a chain whose interfaces are identities equals the full operator,
and with orthonormal interfaces it equals P^T A P; ``local_apply`` equals
``local_matrix`` times the vector; ``dot`` of two rank-1
trains is the product of the factor inner products; the unfolding singular
values of a random train vanish beyond its ranks.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np


def full_vec(cores: Sequence[np.ndarray]) -> np.ndarray:
    out = np.ones((1, 1))
    for c in cores:
        r0, n, r1 = c.shape
        out = (out @ c.reshape(r0, n * r1)).reshape(-1, r1)
    return out.reshape(-1)


def full_mat(cores: Sequence[np.ndarray]) -> np.ndarray:
    out = np.ones((1, 1, 1))          # [rows, cols, r]
    for c in cores:
        R0, m, n, R1 = c.shape
        rows, cols, _ = out.shape
        t = np.einsum("abr,rijs->aibjs", out, c)
        out = t.reshape(rows * m, cols * n, R1)
    return out[:, :, 0]


def matvec(A_cores, x_cores) -> np.ndarray:
    return full_mat(A_cores) @ full_vec(x_cores)


def dot(a_cores, b_cores) -> float:
    return float(full_vec(a_cores) @ full_vec(b_cores))


def unfolding_svals(x: np.ndarray, modes: Sequence[int], k: int) -> np.ndarray:
    """Singular values of the unfolding (modes[:k]) x (modes[k:])."""
    left = int(np.prod(modes[:k]))
    return np.linalg.svd(x.reshape(left, -1), compute_uv=False)


def round_error_bound(x_full: np.ndarray, y_full: np.ndarray) -> float:
    """Relative Frobenius error ||x - y|| / ||x||."""
    return float(np.linalg.norm(x_full - y_full) / np.linalg.norm(x_full))


def left_orthonormal(cores, k: int) -> bool:
    """Is the product of cores[:k] an orthonormal column set?"""
    if k == 0:
        return True
    part = np.ones((1, 1))
    for c in cores[:k]:
        r0, n, r1 = c.shape
        part = (part @ c.reshape(r0, n * r1)).reshape(-1, r1)
    g = part.T @ part
    return bool(np.allclose(g, np.eye(g.shape[0]), atol=1e-10))


def _partial(cores):
    """Dense matrix of a partial train: rows = modes, cols = open bond."""
    part = np.ones((1, 1))
    for c in cores:
        r0, n, r1 = c.shape
        part = (part @ c.reshape(r0, n * r1)).reshape(-1, r1)
    return part


def _partial_right(cores):
    """Dense matrix of a right partial train: rows = open bond, cols = modes."""
    part = np.ones((1, 1))
    for c in reversed(cores):
        r0, n, r1 = c.shape
        part = (c.reshape(r0 * n, r1) @ part).reshape(r0, -1)
    return part


def _partial_mat(cores):
    """Dense tensor of a left partial TT matrix: [rows, cols, open bond]."""
    out = np.ones((1, 1, 1))
    for c in cores:
        R0, m, n, R1 = c.shape
        rows, cols, _ = out.shape
        out = np.einsum("abr,rijs->aibjs", out, c).reshape(rows * m, cols * n, R1)
    return out


def _partial_mat_right(cores):
    """Dense tensor of a right partial TT matrix: [open bond, rows, cols]."""
    out = np.ones((1, 1, 1))
    for c in reversed(cores):
        R0, m, n, R1 = c.shape
        _, rows, cols = out.shape
        out = np.einsum("rijs,sab->riajb", c, out).reshape(R0, m * rows, n * cols)
    return out


def left_interface(x_cores, A_cores, k: int) -> np.ndarray:
    """Phi_L[a, b, a'] = sum X_<k[rows, a] A_<k[rows, cols, b] X_<k[cols, a']."""
    if k == 0:
        return np.ones((1, 1, 1))
    X = _partial(x_cores[:k])
    A = _partial_mat(A_cores[:k])
    return np.einsum("ra,rcb,cd->abd", X, A, X)


def right_interface(x_cores, A_cores, k: int) -> np.ndarray:
    """Phi_R[a, b, a'] = sum X_>k[a, rows] A_>k[b, rows, cols] X_>k[a', cols]."""
    d = len(x_cores)
    if k == d - 1:
        return np.ones((1, 1, 1))
    X = _partial_right(x_cores[k + 1:])
    A = _partial_mat_right(A_cores[k + 1:])
    return np.einsum("ar,brc,dc->abd", X, A, X)


def local_matrix(phiL: np.ndarray, Ak: np.ndarray, phiR: np.ndarray) -> np.ndarray:
    """Dense local operator on x[a, i, c] (row-major):
    sum_{b, b'} PhiL[:, b, :] (x) A_k[b, :, :, b'] (x) PhiR[:, b', :]."""
    rL, RL, _ = phiL.shape
    R0, m, n, R1 = Ak.shape
    rR, RR, _ = phiR.shape
    assert RL == R0 and RR == R1
    out = np.zeros((rL * m * rR, rL * n * rR))
    for b in range(R0):
        for bp in range(R1):
            out += np.kron(np.kron(phiL[:, b, :], Ak[b, :, :, bp]), phiR[:, bp, :])
    return out


def local_apply(phiL: np.ndarray, Ak: np.ndarray, phiR: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The local operator applied to x[a', j, c'] without forming it:
    y[a, i, c] = sum PhiL[a, b, a'] A_k[b, i, j, b'] PhiR[c, b', c'] x[a', j, c']."""
    rL = phiL.shape[0]
    n = Ak.shape[2]
    rR = phiR.shape[0]
    X = x.reshape(rL, n, rR)
    y = np.einsum("aBp,pjc->aBjc", phiL, X)          # contract a'
    y = np.einsum("aBjc,Bijd->aidc", y, Ak)          # contract b, j
    y = np.einsum("aidc,edc->aie", y, phiR)          # contract b', c'
    return y.reshape(-1)


def qtt_of_function(values: np.ndarray, tol: float = 1e-12) -> List[np.ndarray]:
    """TT-SVD of a length-2^l vector reshaped to 2 x ... x 2 (for rank pins)."""
    l = int(round(np.log2(values.size)))
    t = values.reshape((2,) * l)
    nrm = np.linalg.norm(values)
    delta = tol * nrm / np.sqrt(max(l - 1, 1))
    cores = []
    r = 1
    rest = t.reshape(1, -1)
    for k in range(l - 1):
        mat = rest.reshape(r * 2, -1)
        u, s, vt = np.linalg.svd(mat, full_matrices=False)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
        keep = max(1, int(np.sum(tail > delta)))
        cores.append(u[:, :keep].reshape(r, 2, keep))
        rest = s[:keep, None] * vt[:keep]
        r = keep
    cores.append(rest.reshape(r, 2, 1))
    return cores
