"""Dense (sparse-matrix) operators H, S, F for tiny grids, three ways.

TEST INFRASTRUCTURE ONLY (see the package docstring).

1. ``equation_operators``: rows written out from the cell equation
   (eq. Discretized_kNTE) and the vacuum boundary equations
   (eq. discreteBCs).  The equation of cell c for direction l sits at the row
   of c's outgoing vertex; a boundary equation psi = 0 sits at its inflow
   face node.  Optionally, periodic axes: the inflow-face row becomes
   psi(node) = psi(opposite-face node) (an infinite-medium mode the paper
   does not have; it gives the closed-form pins at any grid size).
2. ``appendix_cell_rows``: the cell rows rebuilt from the appendix
   matricization (difference matrix D_x, averaging matrix S_x, Kronecker
   products, zeroth angular moment for isotropic scattering).
3. ``tt_form_operators``: the paper's per-octant Kronecker sums of Section
   3.1 (differentiation matrices D^+-, interpolation matrices Ip^+-, Ip_noBC,
   angular matrices C_o (x) diag, integral matrix, energy factors).
   Readings used: the integral matrix couples every row of octant o to the
   directions of *all* octants (the cell equation sums over all L
   directions); the energy factor of F is chi nu_sigma_f^T and of S is the
   scattering matrix; a row of octant o takes the material of the cell whose
   equation it is (row i -> cell i for a positive cosine, cell i+1 for a
   negative one, clamped to the grid at face rows).

``k_dominant`` is the brute-force generalized eigensolve: the largest
eigenvalue of (H - S)^{-1} F.

Pins (tests/test_oracle_sweep.py, tests/test_oracle_pins.py): the three
assemblies agree row by row; the boundary-row count is the appendix's; the
equation-row H equals the sweep; one LU step equals the sweep checker's
step; with periodic faces (a homogeneous infinite medium) one step from a
constant flux gives k_1 = k_0 sigma_s/sigma_t + nu_sigma_f/sigma_t and a
constant flux, and the brute-force k is nu_sigma_f/(sigma_t - sigma_s) (one
group) or nu_sigma_f^T (diag sigma_t - Sigma_s)^{-1} chi (several groups).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _grid(wl):
    n = wl.n
    return n, n - 1, 1.0 / (n - 1)


def _node(n, k, j, i):
    return (k * n + j) * n + i


def equation_operators(wl, periodic=None):
    """H, S, F (CSR) in the equation-row arrangement, unknowns psi[g,l,k,j,i].

    Node counts and spacings may differ per axis (the cell equation carries
    Delta x_i, Delta y_j, Delta z_k).  ``periodic`` (per axis z, y, x;
    default: ``wl.periodic``) replaces the vacuum row psi = 0 of an
    incoming-face node on that axis by
    psi(node) - psi(node on the opposite face) = 0.  A node on several
    incoming faces takes the condition of the x face first, then y, then z.
    """
    nz, ny, nx = (wl.axis_nodes(ax) for ax in range(3))
    hz, hy, hx = (wl.axis_spacing(ax) for ax in range(3))
    G, L = wl.G, wl.L
    if periodic is None:
        periodic = getattr(wl, "periodic", (False, False, False))
    per_z, per_y, per_x = (bool(p) for p in periodic)
    N = nz * ny * nx
    node = lambda k, j, i: (k * ny + j) * nx + i
    mat = wl.cell_material()
    q = wl.quad
    Hr, Hc, Hv = [], [], []
    Sr, Sc, Sv = [], [], []
    Fr, Fc, Fv = [], [], []
    for g in range(G):
        for l in range(L):
            base = (g * L + l) * N
            mu, eta, xi = q.mu[l], q.eta[l], q.xi[l]
            i_in = 0 if mu > 0 else nx - 1
            j_in = 0 if eta > 0 else ny - 1
            k_in = 0 if xi > 0 else nz - 1
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        if i == i_in or j == j_in or k == k_in:
                            r = base + node(k, j, i)
                            Hr.append(r); Hc.append(r); Hv.append(1.0)
                            if i == i_in:
                                opp = node(k, j, nx - 1 - i) if per_x else None
                            elif j == j_in:
                                opp = node(k, ny - 1 - j, i) if per_y else None
                            else:
                                opp = node(nz - 1 - k, j, i) if per_z else None
                            if opp is not None:
                                Hr.append(r); Hc.append(base + opp); Hv.append(-1.0)
            # cell equations, all cells of this (g, l) at once; cell c = (ck, cj, ci)
            # (1-based) sits at the row of its outgoing vertex
            ck, cj, ci = np.meshgrid(np.arange(1, nz), np.arange(1, ny), np.arange(1, nx),
                                     indexing="ij")
            ck, cj, ci = ck.ravel(), cj.ravel(), ci.ravel()
            ok = ck if xi > 0 else ck - 1
            oj = cj if eta > 0 else cj - 1
            oi = ci if mu > 0 else ci - 1
            rows = base + node(ok, oj, oi)
            m = mat[ck - 1, cj - 1, ci - 1]
            st = wl.sigma_t[m, g]
            verts = [(kk, jj, ii) for kk in (0, 1) for jj in (0, 1) for ii in (0, 1)]
            for dk, dj, di in verts:
                # vertex (ck - 1 + dk, cj - 1 + dj, ci - 1 + di)
                cols = base + node(ck - 1 + dk, cj - 1 + dj, ci - 1 + di)
                v = st / 8.0
                v = v + mu / (4 * hx) * (1.0 if di else -1.0)
                v = v + eta / (4 * hy) * (1.0 if dj else -1.0)
                v = v + xi / (4 * hz) * (1.0 if dk else -1.0)
                Hr.append(rows); Hc.append(cols); Hv.append(np.broadcast_to(v, rows.shape))
            for gp in range(G):
                ss = wl.sigma_s[m, g, gp] / 8.0
                ff = wl.chi[g] * wl.nu_sigma_f[m, gp] / 8.0
                for dk, dj, di in verts:
                    vnode = node(ck - 1 + dk, cj - 1 + dj, ci - 1 + di)
                    for lp in range(L):
                        cols = (gp * L + lp) * N + vnode
                        if np.any(ss != 0.0):
                            Sr.append(rows); Sc.append(cols); Sv.append(ss * q.w[lp])
                        if np.any(ff != 0.0):
                            Fr.append(rows); Fc.append(cols); Fv.append(ff * q.w[lp])
    T = G * L * N
    def mk(r, c, v):
        if not r:
            return sp.csr_matrix((T, T))
        rr = np.concatenate([np.atleast_1d(x).ravel() for x in r]).astype(np.int64)
        cc = np.concatenate([np.atleast_1d(x).ravel() for x in c]).astype(np.int64)
        vv = np.concatenate([np.broadcast_to(np.asarray(x, dtype=float), np.shape(np.atleast_1d(rx))).ravel()
                             for x, rx in zip(v, r)])
        return sp.csr_matrix((vv, (rr, cc)), shape=(T, T))
    return mk(Hr, Hc, Hv), mk(Sr, Sc, Sv), mk(Fr, Fc, Fv)


def _diff_avg(n, h):
    """Appendix difference and averaging matrices, both M x (M+1)."""
    M = n - 1
    D = np.zeros((M, n))
    Sx = np.zeros((M, n))
    for c in range(M):
        D[c, c], D[c, c + 1] = -1.0, 1.0
        Sx[c, c] = Sx[c, c + 1] = 0.5
    return D / h, Sx


def appendix_cell_rows(wl):
    """Cell rows of H, S, F from the appendix Kronecker form.

    Returns CSR matrices with G*L*M^3 rows (cell (ck,cj,ci) -> row
    ((g*L + l)*M + ck-1)*M^2 + ...), columns over all unknowns.
    """
    n, M, h = _grid(wl)
    G, L = wl.G, wl.L
    q = wl.quad
    D, Sx = _diff_avg(n, h)
    Ssp, Dsp = sp.csr_matrix(Sx), sp.csr_matrix(D)
    Kmu = sp.kron(sp.kron(Ssp, Ssp), Dsp)      # S_z (x) S_y (x) dx^{-1} D_x
    Keta = sp.kron(sp.kron(Ssp, Dsp), Ssp)
    Kxi = sp.kron(sp.kron(Dsp, Ssp), Ssp)
    Savg = sp.kron(sp.kron(Ssp, Ssp), Ssp)      # S = S_z (x) S_y (x) S_x
    mat = wl.cell_material().reshape(-1)
    C = M ** 3
    blocksH = [[None] * (G * L) for _ in range(G * L)]
    for g in range(G):
        sig = sp.diags(wl.sigma_t[mat, g])
        for l in range(L):
            blk = q.mu[l] * Kmu + q.eta[l] * Keta + q.xi[l] * Kxi + sig @ Savg
            blocksH[g * L + l][g * L + l] = blk
    for a in range(G * L):
        for b in range(G * L):
            if blocksH[a][b] is None:
                blocksH[a][b] = sp.csr_matrix((C, n ** 3))
    H = sp.bmat(blocksH).tocsr()
    # isotropic scattering: zeroth moment L^0 (weights), replicate with L^{0,+}
    mom = sp.kron(sp.csr_matrix(q.w.reshape(1, -1)), Savg)       # [C, L*N]
    rep = sp.kron(sp.csr_matrix(np.ones((L, 1))), sp.identity(C))  # [L*C, C]
    Srows, Frows = [], []
    for g in range(G):
        rowS, rowF = [], []
        for gp in range(G):
            ss = sp.diags(wl.sigma_s[mat, g, gp])
            ff = sp.diags(wl.chi[g] * wl.nu_sigma_f[mat, gp])
            rowS.append(rep @ ss @ mom)
            rowF.append(rep @ ff @ mom)
        Srows.append(rowS)
        Frows.append(rowF)
    return H, sp.bmat(Srows).tocsr(), sp.bmat(Frows).tocsr()


def cell_row_index(wl):
    """Map appendix cell rows to equation-arrangement rows (outgoing vertex)."""
    n, M, _ = _grid(wl)
    G, L = wl.G, wl.L
    q = wl.quad
    out = np.empty(G * L * M ** 3, dtype=np.int64)
    t = 0
    for g in range(G):
        for l in range(L):
            base = (g * L + l) * n ** 3
            for ck in range(1, n):
                for cj in range(1, n):
                    for ci in range(1, n):
                        ok = ck if q.xi[l] > 0 else ck - 1
                        oj = cj if q.eta[l] > 0 else cj - 1
                        oi = ci if q.mu[l] > 0 else ci - 1
                        out[t] = base + _node(n, ok, oj, oi)
                        t += 1
    return out


# --- the paper's TT-form Kronecker sums (Section 3.1), written densely ---------

def diff_matrix(n, h, positive: bool):
    """D^+ (lower bidiagonal, BC row first) or D^- (upper, BC row last)."""
    D = np.zeros((n, n))
    if positive:
        D[0, 0] = 1.0
        for i in range(1, n):
            D[i, i - 1], D[i, i] = -1.0, 1.0
    else:
        for i in range(n - 1):
            D[i, i], D[i, i + 1] = -1.0, 1.0
        D[n - 1, n - 1] = -1.0
    return D / h


def interp_matrix(n, positive: bool, no_bc: bool = False):
    """Ip^+ / Ip^- and their no-BC variants (the BC row zeroed)."""
    P = np.zeros((n, n))
    if positive:
        P[0, 0] = 1.0
        for i in range(1, n):
            P[i, i - 1] = P[i, i] = 1.0
        if no_bc:
            P[0, 0] = 0.0
    else:
        for i in range(n - 1):
            P[i, i] = P[i, i + 1] = 1.0
        P[n - 1, n - 1] = 1.0
        if no_bc:
            P[n - 1, n - 1] = 0.0
    return 0.5 * P


def _octant_signs(o):
    return bool(o & 1), bool(o & 2), bool(o & 4)   # x, y, z positive


def _row_block_indicator(wl, ax, positive):
    """1D row indicators per block along axis ``ax`` under an octant shift."""
    n, M, _ = _grid(wl)
    ivs = wl.block_intervals(ax)
    out = np.zeros((len(ivs), n))
    for r in range(n):
        cell = r if positive else r + 1
        cell = min(max(cell, 1), M)
        for b, (lo, hi) in enumerate(ivs):
            if lo <= cell <= hi:
                out[b, r] = 1.0
    return out


def tt_form_operators(wl):
    """H, S, F as the per-octant sums of Kronecker products (CSR)."""
    n, M, h = _grid(wl)
    G, L = wl.G, wl.L
    q = wl.quad
    per = L // 8
    I_G = sp.identity(G)
    H = None
    S = None
    F = None

    def add(A, B):
        return B if A is None else A + B

    for o in range(8):
        px, py, pz = _octant_signs(o)
        sel = np.zeros(L)
        sel[o * per:(o + 1) * per] = 1.0
        Qmu, Qeta, Qxi = (sp.diags(sel * q.mu), sp.diags(sel * q.eta), sp.diags(sel * q.xi))
        Dx, Dy, Dz = (sp.csr_matrix(diff_matrix(n, h, s)) for s in (px, py, pz))
        Ix, Iy, Iz = (sp.csr_matrix(interp_matrix(n, s)) for s in (px, py, pz))
        Nx, Ny, Nz = (sp.csr_matrix(interp_matrix(n, s, True)) for s in (px, py, pz))
        H = add(H, sp.kron(sp.kron(sp.kron(sp.kron(I_G, Qmu), Iz), Iy), Dx))
        H = add(H, sp.kron(sp.kron(sp.kron(sp.kron(I_G, Qeta), Iz), Dy), Ix))
        H = add(H, sp.kron(sp.kron(sp.kron(sp.kron(I_G, Qxi), Dz), Iy), Ix))
        Csel = sp.diags(sel)
        Intg = sp.csr_matrix(np.outer(sel, q.w))
        indz = _row_block_indicator(wl, 0, pz)
        indy = _row_block_indicator(wl, 1, py)
        indx = _row_block_indicator(wl, 2, px)
        Bz, By, Bx = wl.block_mat.shape
        for bz in range(Bz):
            for by in range(By):
                for bx in range(Bx):
                    m = wl.block_mat[bz, by, bx]
                    Rz, Ry, Rx = sp.diags(indz[bz]), sp.diags(indy[by]), sp.diags(indx[bx])
                    spat = sp.kron(sp.kron(Rz @ Iz, Ry @ Iy), Rx @ Ix)
                    spatN = sp.kron(sp.kron(Rz @ Nz, Ry @ Ny), Rx @ Nx)
                    H = add(H, sp.kron(sp.kron(sp.diags(wl.sigma_t[m]), Csel), spat))
                    Es = sp.csr_matrix(wl.sigma_s[m])
                    Ef = sp.csr_matrix(np.outer(wl.chi, wl.nu_sigma_f[m]))
                    S = add(S, sp.kron(sp.kron(Es, Intg), spatN))
                    F = add(F, sp.kron(sp.kron(Ef, Intg), spatN))
    return H.tocsr(), S.tocsr(), F.tocsr()


def k_dominant(H, S, F, dense: bool = False) -> float:
    """Largest eigenvalue of (H - S)^{-1} F (the generalized k eigenproblem)."""
    A = (H - S).tocsc()
    if dense:
        ev = scipy.linalg.eigvals(np.linalg.solve(A.toarray(), F.toarray()))
        ev = ev[np.argsort(-np.abs(ev))]
        return float(ev[0].real)
    lu = spla.splu(A)
    op = spla.LinearOperator(A.shape, matvec=lambda x: lu.solve(F @ x), dtype=np.float64)
    ev = spla.eigs(op, k=1, which="LM", tol=1e-14, maxiter=20000, return_eigenvectors=False)
    return float(ev[0].real)
