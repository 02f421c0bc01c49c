"""Transport operators H, S, F as mixed TT/QTT matrices (host setup).

Builds the operators of eq. OpFormkNTE in the chain order
``[energy][angle][z bits][y bits][x bits]`` (the Kronecker order of the
per-octant terms in Section 3.1; the energy core is dropped when G = 1).
Space is QTT (Section 2.2); energy and angle are plain TT cores because the
group and direction counts need not be powers of two.

Per octant o (sign of mu, eta, xi), following Section 3.1:
  H_x^o = I_G (x) Q_mu^o  (x) Ip_z (x) Ip_y (x) D_x
  H_y^o = I_G (x) Q_eta^o (x) Ip_z (x) D_y  (x) Ip_x
  H_z^o = I_G (x) Q_xi^o  (x) D_z  (x) Ip_y (x) Ip_x
  H_s^o = diag(sigma_t) (x) (C_o (x) I) (x) Ip_z (x) Ip_y (x) Ip_x
  S^o   = Sigma_s (x) Intg^o (x) Ip_z,noBC (x) Ip_y,noBC (x) Ip_x,noBC
  F^o   = chi nu_sigma_f^T (x) Intg^o (x) (same)
and each operator is the sum over octants (eq. for F^TT, S^TT and H^QTT).

Readings of under-specified passages:
  * the integral matrix Intg^o has the rows of octant o and the columns of
    every direction, weighted by w (the cell equation sums over all L
    directions);
  * the energy factor of F is chi nu_sigma_f^T and of S the scattering
    matrix (the per-group diagonal factors written in Section 3.1 only make
    sense for one group);
  * heterogeneous media: the row of octant o at node index i along an axis is
    the equation of cell i (positive cosine) or cell i+1 (negative cosine);
    face rows, which carry no cell, take the adjacent cell.  The material
    weights multiply those rows.  A material map made of axis-aligned blocks
    is a small coefficient tensor over (energy, z block, y block, x block);
    its exact TT factors are bridged into each axis by interval indicators.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import qtt
from .qtt import Cores


@dataclasses.dataclass
class Operators:
    H: Cores
    S: Cores
    F: Cores
    cF: Cores           # F^T 1 as a TT vector (fission-rate functional)
    psi0: Cores         # seeded rank-1 initial flux
    modes: List[int]    # mode size per core


def _octant_signs(o):
    return bool(o & 1), bool(o & 2), bool(o & 4)


def _diff(l, h, pos):
    # D^+ = (I - J)/h (lower bidiagonal, BC row first); D^- = (-I + J^T)/h
    return qtt.qtt_bidiag(l, 1.0 / h, -1.0 / h, True) if pos else \
        qtt.qtt_bidiag(l, -1.0 / h, 1.0 / h, False)


def _interp(l, pos, no_bc=False):
    base = qtt.qtt_bidiag(l, 0.5, 0.5, pos)
    if not no_bc:
        return base
    return qtt.tt_sum([base, qtt.qtt_corner(l, pos, -0.5)])


def _diff_nobc(l, h, pos):
    # D^+ without its inflow row (row 0, entry 1/h); D^- without row n-1 (-1/h)
    return qtt.tt_sum([_diff(l, h, pos), qtt.qtt_corner(l, pos, -1.0 / h if pos else 1.0 / h)])


def _row_projector(l, pos):
    # I minus the inflow-row selector e_in e_in^T
    return qtt.tt_sum([qtt.qtt_eye(l), qtt.qtt_corner(l, pos, -1.0)])


def _face_rows(l, h, pos, periodic):
    """(1/h) e_in (e_in - e_out)^T for a periodic axis, (1/h) e_in e_in^T for a
    vacuum one; e_in is node 0 for a positive cosine, node n-1 otherwise."""
    rows = qtt.qtt_corner(l, pos, 1.0 / h)
    if not periodic:
        return rows
    return qtt.tt_sum([rows, qtt.qtt_outer(l, pos, not pos, -1.0 / h)])


def _row_intervals(wl, ax, pos):
    """Node-row interval of every block along axis ``ax`` for one octant sign.

    Row i holds the equation of cell i (pos) or cell i+1 (neg); the face row
    (0 for pos, n-1 for neg) joins the block of the adjacent cell.
    """
    n = wl.axis_nodes(ax)
    M = n - 1
    out = []
    for lo, hi in wl.block_intervals(ax):
        if pos:
            a = 0 if lo == 1 else lo
            b = hi
        else:
            a = lo - 1
            b = n - 1 if hi == M else hi - 1
        out.append((a, b))
    return out


def _coef_tt(coef: np.ndarray):
    """Exact TT factors of the block coefficient tensor [E, Bz, By, Bx]."""
    cores = qtt.tt_svd(coef, tol=1e-15)
    e = cores[0][0]           # [E, a1]
    return e, cores[1], cores[2], cores[3][:, :, 0]


def _material_term(wl, o, energy_mats: np.ndarray, no_bc: bool,
                   collision: bool = False) -> Cores:
    """sum_blocks E[mat(b)] (x) angle (x) R_z P_z (x) R_y P_y (x) R_x P_x.

    ``energy_mats[m]`` is the G x G energy factor of material m; the angle
    factor is C_o (x) I for H (no_bc False, or ``collision``) or Intg^o for
    S, F (no_bc True).
    """
    G, L = wl.G, wl.L
    per = L // 8
    sel = np.zeros(L)
    sel[o * per:(o + 1) * per] = 1.0
    angle = np.outer(sel, wl.quad.w) if (no_bc and not collision) else np.diag(sel)
    Bz, By, Bx = wl.block_mat.shape
    coef = np.zeros((G * G, Bz, By, Bx))
    for bz in range(Bz):
        for by in range(By):
            for bx in range(Bx):
                coef[:, bz, by, bx] = energy_mats[wl.block_mat[bz, by, bx]].reshape(-1)
    e, cz, cy, cx = _coef_tt(coef)
    a1 = e.shape[1]
    cores: Cores = []
    if G > 1:
        cores.append(e.reshape(1, G, G, a1))
        cores.append(np.einsum("ab,mn->amnb", np.eye(a1), angle))
    else:
        cores.append(np.einsum("b,mn->mnb", e[0], angle)[None])
    signs = _octant_signs(o)
    for ax, c in zip((0, 1, 2), (cz, cy, cx)):
        pos = signs[2 - ax]                  # axis 0 is z (sign bit 4), 2 is x (bit 1)
        l = wl.axis_bits(ax)
        P = _interp(l, pos, no_bc)
        blocks = []
        for (a, b) in _row_intervals(wl, ax, pos):
            R = qtt.vec_to_diag(qtt.qtt_interval(l, a, b))
            blocks.append(qtt.mat_mat(R, P))
        if ax == 2:
            c = c[:, :, None]
        cores.extend(qtt.bridge_segment(c, blocks))
    return cores


def _energy_angle(wl, Qdiag) -> Cores:
    G = wl.G
    out = []
    if G > 1:
        out += qtt.single(np.eye(G))
    out += qtt.single(np.diag(Qdiag))
    return out


def octant_terms(wl, o):
    """The streaming and collision terms of H for one octant (list of TTs)."""
    lz, ly, lx = (wl.axis_bits(ax) for ax in range(3))
    hz, hy, hx = (wl.axis_spacing(ax) for ax in range(3))
    px, py, pz = _octant_signs(o)
    per = wl.L // 8
    sel = np.zeros(wl.L)
    sel[o * per:(o + 1) * per] = 1.0
    q = wl.quad
    Ix, Iy, Iz = _interp(lx, px), _interp(ly, py), _interp(lz, pz)
    Dx, Dy, Dz = _diff(lx, hx, px), _diff(ly, hy, py), _diff(lz, hz, pz)
    terms = [
        qtt.kron_chain([_energy_angle(wl, sel * q.mu), Iz, Iy, Dx]),
        qtt.kron_chain([_energy_angle(wl, sel * q.eta), Iz, Dy, Ix]),
        qtt.kron_chain([_energy_angle(wl, sel * q.xi), Dz, Iy, Ix]),
        _material_term(wl, o, np.stack([np.diag(s) for s in wl.sigma_t]), False),
    ]
    return terms


def octant_terms_explicit_faces(wl, o):
    """Octant o's rows of H with explicit face rows (used when an axis is periodic).

    The cell rows are the terms of ``octant_terms`` with every 1D factor's
    inflow row removed (so they vanish on the inflow faces).  Each inflow-face
    node then gets one row, taken from the x face first, then y, then z:
    psi(node) - psi(opposite node) = 0 on a periodic axis, psi(node) = 0 on a
    vacuum one (both scaled by 1/h).  For vacuum axes this has the same
    solutions as ``octant_terms``, whose face rows are a two-dimensional
    transport problem with no source.
    """
    lz, ly, lx = (wl.axis_bits(ax) for ax in range(3))
    hz, hy, hx = (wl.axis_spacing(ax) for ax in range(3))
    px, py, pz = _octant_signs(o)
    per_z, per_y, per_x = (bool(p) for p in wl.periodic)
    per = wl.L // 8
    sel = np.zeros(wl.L)
    sel[o * per:(o + 1) * per] = 1.0
    q = wl.quad
    Ix, Iy, Iz = _interp(lx, px, True), _interp(ly, py, True), _interp(lz, pz, True)
    Dx, Dy, Dz = _diff_nobc(lx, hx, px), _diff_nobc(ly, hy, py), _diff_nobc(lz, hz, pz)
    Px, Py = _row_projector(lx, px), _row_projector(ly, py)
    Ey, Ez = qtt.qtt_eye(ly), qtt.qtt_eye(lz)
    return [
        qtt.kron_chain([_energy_angle(wl, sel * q.mu), Iz, Iy, Dx]),
        qtt.kron_chain([_energy_angle(wl, sel * q.eta), Iz, Dy, Ix]),
        qtt.kron_chain([_energy_angle(wl, sel * q.xi), Dz, Iy, Ix]),
        _material_term(wl, o, np.stack([np.diag(s) for s in wl.sigma_t]), True, collision=True),
        qtt.kron_chain([_energy_angle(wl, sel), Ez, Ey, _face_rows(lx, hx, px, per_x)]),
        qtt.kron_chain([_energy_angle(wl, sel), Ez, _face_rows(ly, hy, py, per_y), Px]),
        qtt.kron_chain([_energy_angle(wl, sel), _face_rows(lz, hz, pz, per_z), Py, Px]),
    ]


def _round(cores, tol):
    return qtt.tt_round_host(cores, tol)


# The angle factor of every term is diagonal in H (C_o (x) I, Q_mu^o, ...) and
# of the form a (x) w^T in S and F (Intg^o = sel_o w^T, the same w for every
# octant).  Rounding sums of such terms with the L x L angle mode stored in
# full would factor L^2-long unfoldings; the compressed forms below carry only
# the L row entries and are exact, so the rounded operator is the same.
def _angle_index(wl) -> int:
    return 1 if wl.G > 1 else 0


def _squeeze_angle(cores: Cores, wl, kind: str) -> Cores:
    k = _angle_index(wl)
    c = cores[k]
    if kind == "diag":
        a = np.einsum("aiib->aib", c)
        assert np.array_equal(c, np.einsum("aib,ij->aijb", a, np.eye(c.shape[1]))), "angle not diagonal"
    else:
        w = wl.quad.w
        a = c[:, :, 0, :] / w[0]
        assert np.allclose(c, np.einsum("aib,j->aijb", a, w), rtol=1e-14, atol=0), "angle not a w^T"
    out = list(cores)
    out[k] = a[:, :, None, :]
    return out


def _expand_angle(cores: Cores, wl, kind: str) -> Cores:
    k = _angle_index(wl)
    a = cores[k][:, :, 0, :]
    out = list(cores)
    if kind == "diag":
        out[k] = np.einsum("aib,ij->aijb", a, np.eye(a.shape[1]))
    else:
        out[k] = np.einsum("aib,j->aijb", a, wl.quad.w)
    return out


def build(wl, tol: float = 1e-13) -> Operators:
    """Assemble H, S, F (each summed over octants and compressed exactly)."""
    H = None
    S = None
    F = None
    Es = np.asarray(wl.sigma_s)
    Ef = np.einsum("g,mh->mgh", wl.chi, wl.nu_sigma_f)
    explicit = any(getattr(wl, "periodic", (False, False, False)))
    for o in range(8):
        terms = octant_terms_explicit_faces(wl, o) if explicit else octant_terms(wl, o)
        Ho = _round(qtt.tt_sum([_squeeze_angle(t, wl, "diag") for t in terms]), tol)
        H = Ho if H is None else _round(qtt.tt_sum([H, Ho]), tol)
        So = _round(_squeeze_angle(_material_term(wl, o, Es, True), wl, "w"), tol)
        S = So if S is None else _round(qtt.tt_sum([S, So]), tol)
        Fo = _round(_squeeze_angle(_material_term(wl, o, Ef, True), wl, "w"), tol)
        F = Fo if F is None else _round(qtt.tt_sum([F, Fo]), tol)
    H = _expand_angle(H, wl, "diag")
    S = _expand_angle(S, wl, "w")
    F = _expand_angle(F, wl, "w")
    cF = [c.sum(axis=1) for c in F]          # F^T 1: sum over the row mode
    cF = qtt.tt_round_host(cF, tol)
    psi0 = []
    if wl.G > 1:
        psi0.append(wl.psi0_energy.reshape(1, -1, 1).copy())
    psi0.append(wl.psi0_angle.reshape(1, -1, 1).copy())
    for ax in range(3):
        for b in range(wl.axis_bits(ax)):
            psi0.append(wl.psi0_bits[ax, b].reshape(1, 2, 1).copy())
    modes = [c.shape[1] for c in psi0]
    return Operators(H, S, F, cF, psi0, modes)


def build_unrounded(wl):
    """The plain sums (no compression); for checking the construction."""
    Es = np.asarray(wl.sigma_s)
    Ef = np.einsum("g,mh->mgh", wl.chi, wl.nu_sigma_f)
    Ht, St, Ft = [], [], []
    explicit = any(getattr(wl, "periodic", (False, False, False)))
    for o in range(8):
        Ht += octant_terms_explicit_faces(wl, o) if explicit else octant_terms(wl, o)
        St.append(_material_term(wl, o, Es, True))
        Ft.append(_material_term(wl, o, Ef, True))
    return qtt.tt_sum(Ht), qtt.tt_sum(St), qtt.tt_sum(Ft)
