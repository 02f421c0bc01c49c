"""Host-side tensor-train containers and exact QTT building blocks (setup only).

Layouts (row-major, last index fastest):
  * TT vector core k:  ``[r_{k-1}, n_k, r_k]``
  * TT matrix core k:  ``[R_{k-1}, m_k, n_k, R_k]`` (m = output/row mode,
    n = input/column mode), the index-paired form of eq. permute and
    eq. TT-matrix-componentwise.

QTT (Section 2.2, "Quantized Tensor Train"): an axis with ``n = 2**l`` nodes
becomes ``l`` cores of mode size 2, most significant bit first, so node
``i = sum_b i_b 2^(l-1-b)``.

The 1D factors of the transport operators are bidiagonal Toeplitz matrices
plus one corner correction.  Their QTT forms are written here in closed form
(a binary carry automaton for the shift, a comparison automaton for interval
indicators) instead of by the TT-SVD of Algorithm TTtoQTT: the result is the
same exact QTT, obtained without a factorization.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

Cores = List[np.ndarray]


# ---------------------------------------------------------------------------
# 1D QTT matrices
# ---------------------------------------------------------------------------

def qtt_eye(l: int) -> Cores:
    return [np.eye(2).reshape(1, 2, 2, 1).copy() for _ in range(l)]


def qtt_bidiag(l: int, a: float, c: float, lower: bool) -> Cores:
    """QTT (rank 2) of ``a*I + c*J`` with J the lower shift (J[i, i-1] = 1),
    or of ``a*I + c*J^T`` when ``lower`` is False.

    Row index i and column index j satisfy i = j + s (lower) or j = i + s
    (upper) with s in {0, 1}; s is the carry entering the least significant
    bit, weighted a for s = 0 and c for s = 1.  The bond between two bit cores
    carries the carry passed from the less to the more significant bit; the
    most significant core admits no overflow.
    """
    def put(core, left, i, j, right, v):
        if lower:
            core[left, i, j, right] += v
        else:
            core[left, j, i, right] += v

    if l == 1:
        core = np.zeros((1, 2, 2, 1))
        for s, wgt in ((0, a), (1, c)):
            for j in range(2):
                t = j + s
                if t < 2:
                    put(core, 0, t, j, 0, wgt)
        return [core]
    cores = []
    first = np.zeros((1, 2, 2, 2))
    for kin in range(2):
        for j in range(2):
            t = j + kin
            if t < 2:
                put(first, 0, t, j, kin, 1.0)
    cores.append(first)
    for _ in range(l - 2):
        mid = np.zeros((2, 2, 2, 2))
        for kin in range(2):
            for j in range(2):
                t = j + kin
                put(mid, t // 2, t % 2, j, kin, 1.0)
        cores.append(mid)
    last = np.zeros((2, 2, 2, 1))
    for s, wgt in ((0, a), (1, c)):
        for j in range(2):
            t = j + s
            put(last, t // 2, t % 2, j, 0, wgt)
    cores.append(last)
    return cores


def qtt_corner(l: int, first: bool, value: float) -> Cores:
    """``value * e e^T`` for e the first (node 0) or last (node n-1) basis vector."""
    b = 0 if first else 1
    cores = []
    for t in range(l):
        c = np.zeros((1, 2, 2, 1))
        c[0, b, b, 0] = value if t == 0 else 1.0
        cores.append(c)
    return cores


def qtt_outer(l: int, row_first: bool, col_first: bool, value: float) -> Cores:
    """``value * e_a e_b^T`` for e_a, e_b each the first (node 0) or last
    (node n-1) basis vector: one nonzero per bit core (rank 1)."""
    a = 0 if row_first else 1
    b = 0 if col_first else 1
    cores = []
    for t in range(l):
        c = np.zeros((1, 2, 2, 1))
        c[0, a, b, 0] = value if t == 0 else 1.0
        cores.append(c)
    return cores


def qtt_interval(l: int, lo: int, hi: int) -> Cores:
    """QTT vector (cores [r, 2, r']) of the indicator of lo <= i <= hi.

    Most-significant-bit-first comparison automaton: the state records
    whether the prefix of i is equal to / greater than the prefix of ``lo``
    and equal to / less than the prefix of ``hi``; states that already left
    the interval are dropped, leaving at most 4 live states.
    """
    n = 1 << l
    if hi < lo:
        return [np.zeros((1, 2, 1)) for _ in range(l)]
    lo, hi = max(lo, 0), min(hi, n - 1)
    states = [(0, 0)]   # (cmp_lo: 0 eq / 1 gt, cmp_hi: 0 eq / 1 lt)
    cores = []
    for t in range(l):
        bit_lo = (lo >> (l - 1 - t)) & 1
        bit_hi = (hi >> (l - 1 - t)) & 1
        nxt = []
        trans = []
        for si, (cl, ch) in enumerate(states):
            for b in range(2):
                if cl == 0:
                    if b < bit_lo:
                        continue
                    ncl = 1 if b > bit_lo else 0
                else:
                    ncl = 1
                if ch == 0:
                    if b > bit_hi:
                        continue
                    nch = 1 if b < bit_hi else 0
                else:
                    nch = 1
                st = (ncl, nch)
                if st not in nxt:
                    nxt.append(st)
                trans.append((si, b, nxt.index(st)))
        last = t == l - 1
        core = np.zeros((len(states), 2, 1 if last else len(nxt)))
        for si, b, so in trans:
            core[si, b, 0 if last else so] += 1.0
        cores.append(core)
        states = nxt
    return cores


def vec_to_diag(cores: Cores) -> Cores:
    """TT vector -> TT matrix of diag(v)."""
    out = []
    for c in cores:
        r, n, rr = c.shape
        d = np.zeros((r, n, n, rr))
        for i in range(n):
            d[:, i, i, :] = c[:, i, :]
        out.append(d)
    return out


def mat_mat(A: Cores, B: Cores) -> Cores:
    """Exact product of TT matrices (A @ B), core-wise; ranks multiply."""
    out = []
    for a, b in zip(A, B):
        Ra, m, k, Ra2 = a.shape
        Rb, k2, n, Rb2 = b.shape
        assert k == k2
        c = np.einsum("aikb,ckjd->acijbd", a, b).reshape(Ra * Rb, m, n, Ra2 * Rb2)
        out.append(c)
    return out


def scale(cores: Cores, s: float) -> Cores:
    out = [c.copy() for c in cores]
    out[0] = out[0] * s
    return out


def tt_sum(terms: Sequence[Cores]) -> Cores:
    """Sum of TT tensors (vectors or matrices) by block concatenation."""
    terms = [t for t in terms if t is not None]
    if len(terms) == 1:
        return [c.copy() for c in terms[0]]
    d = len(terms[0])
    out = []
    for k in range(d):
        cs = [t[k] for t in terms]
        mode = cs[0].shape[1:-1]
        lr = [c.shape[0] for c in cs]
        rr = [c.shape[-1] for c in cs]
        if d == 1:
            out.append(sum(cs))
            continue
        if k == 0:
            L = 1
            R = sum(rr)
        elif k == d - 1:
            L = sum(lr)
            R = 1
        else:
            L, R = sum(lr), sum(rr)
        core = np.zeros((L,) + mode + (R,))
        lo = ro = 0
        for c in cs:
            a, b = c.shape[0], c.shape[-1]
            ls = slice(0, 1) if k == 0 else slice(lo, lo + a)
            rs = slice(0, 1) if k == d - 1 else slice(ro, ro + b)
            core[(ls,) + (slice(None),) * len(mode) + (rs,)] += c
            lo += a
            ro += b
        out.append(core)
    return out


def kron_chain(factors: Sequence[Cores]) -> Cores:
    """Concatenate the core lists of factors acting on consecutive modes."""
    out = []
    for f in factors:
        out.extend(f)
    return out


def single(mat: np.ndarray) -> Cores:
    """A plain (non-quantized) operator core: one mode of size n."""
    m, n = mat.shape
    return [mat.reshape(1, m, n, 1).astype(np.float64)]


def bridge_segment(coef: np.ndarray, blocks: Sequence[Cores]) -> Cores:
    """Segment sum_b coef[a, b, a'] * blocks[b] with open bonds a (left), a' (right).

    ``blocks[b]`` is a TT matrix (rank-1 ends) over the segment's modes.  The
    coefficient enters the first core; the right bond index is carried
    through the block-diagonal inner cores and closed by the last core.
    """
    A, B, A2 = coef.shape
    l = len(blocks[0])
    if l == 1:
        c0 = blocks[0][0]
        core = np.zeros((A,) + c0.shape[1:-1] + (A2,))
        for b in range(B):
            core += np.einsum("ij,mn->imnj", coef[:, b, :], blocks[b][0][0, :, :, 0])
        return [core]
    widths = []
    for b in range(B):
        widths.append([blocks[b][t].shape[-1] for t in range(l - 1)])
    out = []
    # first core: [A][m][n][sum_b A2 * r_b1]
    tot = sum(A2 * w[0] for w in widths)
    m, n = blocks[0][0].shape[1:3]
    first = np.zeros((A, m, n, tot))
    off = 0
    for b in range(B):
        c = blocks[b][0][0]            # [m, n, r1]
        r1 = c.shape[-1]
        for a2 in range(A2):
            first[:, :, :, off:off + r1] += np.einsum("a,mnr->amnr", coef[:, b, a2], c)
            off += r1
    out.append(first)
    for t in range(1, l - 1):
        tl = sum(A2 * w[t - 1] for w in widths)
        tr = sum(A2 * w[t] for w in widths)
        m, n = blocks[0][t].shape[1:3]
        core = np.zeros((tl, m, n, tr))
        ol = orr = 0
        for b in range(B):
            c = blocks[b][t]
            for a2 in range(A2):
                core[ol:ol + c.shape[0], :, :, orr:orr + c.shape[-1]] = c
                ol += c.shape[0]
                orr += c.shape[-1]
        out.append(core)
    tl = sum(A2 * w[l - 2] for w in widths)
    m, n = blocks[0][l - 1].shape[1:3]
    last = np.zeros((tl, m, n, A2))
    ol = 0
    for b in range(B):
        c = blocks[b][l - 1]          # [r, m, n, 1]
        for a2 in range(A2):
            last[ol:ol + c.shape[0], :, :, a2] = c[:, :, :, 0]
            ol += c.shape[0]
    out.append(last)
    return out


# ---------------------------------------------------------------------------
# Host reconstruction helpers used by setup self-checks
# ---------------------------------------------------------------------------

def ranks(cores: Cores) -> List[int]:
    return [cores[0].shape[0]] + [c.shape[-1] for c in cores]


def tt_svd(tensor: np.ndarray, tol: float = 1e-14) -> Cores:
    """Exact-to-``tol`` TT decomposition of a small dense tensor (setup only).

    Sequential truncated SVDs of the unfoldings (the decomposition step of
    Algorithm TTtoQTT), with the relative Frobenius threshold split evenly
    over the d-1 bonds.
    """
    shape = tensor.shape
    d = len(shape)
    nrm = np.linalg.norm(tensor)
    delta = tol * nrm / np.sqrt(max(d - 1, 1))
    cores = []
    r = 1
    rest = tensor.reshape(1, -1)
    for k in range(d - 1):
        mat = rest.reshape(r * shape[k], -1)
        u, s, vt = _svd(mat)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
        keep = max(1, int(np.sum(tail > delta)))
        cores.append(u[:, :keep].reshape(r, shape[k], keep))
        rest = s[:keep, None] * vt[:keep]
        r = keep
    cores.append(rest.reshape(r, shape[-1], 1))
    return cores


def _as_vec(cores: Cores):
    shapes = [c.shape for c in cores]
    vec = [c.reshape(c.shape[0], -1, c.shape[-1]) for c in cores]
    return vec, shapes


def _from_vec(vec: Cores, shapes) -> Cores:
    out = []
    for c, s in zip(vec, shapes):
        out.append(c.reshape((c.shape[0],) + tuple(s[1:-1]) + (c.shape[-1],)))
    return out


def _svd(m: np.ndarray):
    """Thin SVD; LAPACK's divide-and-conquer driver can fail to converge on
    some matrices, then the QR-iteration driver is used."""
    try:
        return np.linalg.svd(m, full_matrices=False)
    except np.linalg.LinAlgError:
        import scipy.linalg
        return scipy.linalg.svd(m, full_matrices=False, lapack_driver="gesvd")


def tt_round_host(cores: Cores, tol: float, rmax: int = 1 << 30) -> Cores:
    """TT rounding on the host (operator setup only): left-to-right QR
    orthogonalization, then right-to-left truncated SVD with the threshold
    tol * ||X|| / sqrt(d-1) per bond.  Matrix cores are rounded as vector
    cores whose mode is the (row, column) pair."""
    vec, shapes = _as_vec(cores)
    d = len(vec)
    if d == 1:
        return [c.copy() for c in cores]
    vec = [c.copy() for c in vec]
    for k in range(d - 1):
        r0, n, r1 = vec[k].shape
        q, rr = np.linalg.qr(vec[k].reshape(r0 * n, r1))
        vec[k] = q.reshape(r0, n, q.shape[1])
        b, n1, c1 = vec[k + 1].shape
        vec[k + 1] = (rr @ vec[k + 1].reshape(b, n1 * c1)).reshape(rr.shape[0], n1, c1)
    nrm = np.linalg.norm(vec[-1])
    delta = tol * nrm / np.sqrt(d - 1)
    for k in range(d - 1, 0, -1):
        r0, n, r1 = vec[k].shape
        u, s, vt = _svd(vec[k].reshape(r0, n * r1))
        tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
        keep = max(1, min(rmax, int(np.sum(tail > delta))))
        vec[k] = vt[:keep].reshape(keep, n, r1)
        a0, n0, b0 = vec[k - 1].shape
        vec[k - 1] = (vec[k - 1].reshape(a0 * n0, b0) @ (u[:, :keep] * s[:keep])).reshape(
            a0, n0, keep)
    return _from_vec(vec, shapes)
