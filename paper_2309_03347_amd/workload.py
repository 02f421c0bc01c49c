"""Seeded synthetic k-eigenvalue workloads (inputs only).

This module draws every random input that both the device solver and the
CPU checker consume: grid size, discrete-ordinates point set and weights,
block-structured material map, multigroup cross sections, and the factors of
the rank-1 initial flux.  It holds none of the method's arithmetic: no
operator, no sweep, no tensor-train algebra.  Each consumer forms its own
representation (dense arrays, QTT cores) from these plain arrays.

Conventions (shared by every consumer):

* Grid: ``n = 2**l`` nodes per axis on the unit cube, ``M = n - 1`` cells per
  axis, spacing ``1/(n-1)``.  Cells along an axis are numbered ``1..M``; cell
  ``c`` spans nodes ``c-1`` and ``c`` (appendix, diamond-difference section).
* Unknown ordering ``psi[g, l, k, j, i]``: energy slowest, then direction,
  then z, y, x node (appendix, matricization of the equations).
* Directions are grouped in eight octant blocks ordered as in the paper's
  ordinate ordering: octant ``o = bx + 2*by + 4*bz`` where ``b = 1`` means the
  cosine along that axis is positive.  Every octant holds the same
  ``L/8`` magnitude triples with that octant's signs; direction index is
  ``ell = o * (L // 8) + m``.
* Materials: each axis is split into blocks of consecutive cells by
  ``cuts`` (list of cell indices where a new block starts); ``block_mat``
  (shape ``[Bz, By, Bx]``) gives the material of every block.
* Cross sections per material ``m``: ``sigma_t[m, g]``, ``sigma_s[m, g, gp]``
  (scatter from group ``gp`` into group ``g``), ``nu_sigma_f[m, g]``;
  one fission spectrum ``chi[g]`` with ``sum(chi) == 1``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Level-symmetric (LQn) first direction cosine for each S_N order.  With it
# the cosines of the set follow mu_i^2 = mu_1^2 + (i-1) * 2 (1 - 3 mu_1^2)/(N-2)
# and every point (mu_i, mu_j, mu_k) with i + j + k = N/2 + 2 lies on the
# unit sphere.
_LQN_MU1 = {2: 1.0 / math.sqrt(3.0), 4: 0.3500212, 6: 0.2666355,
            8: 0.2182179, 16: 0.1389568}


@dataclasses.dataclass
class Quadrature:
    """Discrete ordinates: signed cosines and weights, length L each."""
    mu: np.ndarray
    eta: np.ndarray
    xi: np.ndarray
    w: np.ndarray

    @property
    def L(self) -> int:
        return int(self.mu.shape[0])


@dataclasses.dataclass
class Workload:
    """One seeded k-eigenvalue instance (plain arrays only)."""
    name: str
    l: int                      # bits per spatial axis, n = 2**l nodes
    G: int                      # energy groups
    quad: Quadrature
    cuts: List[List[int]]       # per axis (z, y, x): first cell of blocks 2..B
    block_mat: np.ndarray       # int [Bz, By, Bx]
    sigma_t: np.ndarray         # [Mat, G]
    sigma_s: np.ndarray         # [Mat, G, G]  (g <- gp)
    nu_sigma_f: np.ndarray      # [Mat, G]
    chi: np.ndarray             # [G]
    psi0_energy: np.ndarray     # [G]
    psi0_angle: np.ndarray      # [L]
    psi0_bits: np.ndarray       # [3, l, 2]  (z, y, x; most significant bit first)
    rmax: int
    tol: float
    tol_k: float
    seed: int
    boundary: str = "vacuum"    # "vacuum", or "reflective" (lagged mirror faces, sweep checker only)
    periodic: tuple = (False, False, False)   # per axis (z, y, x): inflow face = opposite face
    l_axes: Optional[tuple] = None            # per axis (z, y, x) bits; None: l on every axis
    lengths: tuple = (1.0, 1.0, 1.0)          # per axis (z, y, x) extent of the box

    @property
    def n(self) -> int:
        return 1 << self.l

    @property
    def M(self) -> int:
        return self.n - 1

    @property
    def L(self) -> int:
        return self.quad.L

    def axis_bits(self, ax: int) -> int:
        return self.l if self.l_axes is None else int(self.l_axes[ax])

    def axis_nodes(self, ax: int) -> int:
        return 1 << self.axis_bits(ax)

    def axis_spacing(self, ax: int) -> float:
        return float(self.lengths[ax]) / (self.axis_nodes(ax) - 1)

    @property
    def shape(self):
        """Node counts per axis (z, y, x)."""
        return tuple(self.axis_nodes(ax) for ax in range(3))

    @property
    def n_nodes(self) -> int:
        nz, ny, nx = self.shape
        return nz * ny * nx

    def cell_material(self) -> np.ndarray:
        """Material id of every cell, int array [Mz, My, Mx] indexed (cz-1, cy-1, cx-1)."""
        idx = []
        for ax in range(3):
            b = np.zeros(self.axis_nodes(ax) - 1, dtype=np.int64)
            for c in self.cuts[ax]:
                b[c - 1:] += 1
            idx.append(b)
        return self.block_mat[np.ix_(idx[0], idx[1], idx[2])]

    def block_intervals(self, ax: int):
        """Inclusive 1-based cell interval of every block along axis ``ax``."""
        starts = [1] + list(self.cuts[ax])
        ends = [s - 1 for s in self.cuts[ax]] + [self.axis_nodes(ax) - 1]
        return list(zip(starts, ends))


def level_symmetric(N: int) -> Quadrature:
    """LQn point set of order N in the paper's octant order, with LQn weights.

    The points of one octant fall into classes (the multiset of their three
    cosine indices); every point of a class gets the same weight, and the
    class weights make the set integrate mu^(2m) exactly for m < N/2 (the
    even-moment conditions that define the level-symmetric weights; they
    reproduce the published LQn values, e.g. 0.1209877, 0.0907407 and
    0.0925926 for S8 with the octant normalized to 1).  Weights sum to 1 over
    all L directions.
    """
    if N not in _LQN_MU1:
        raise ValueError(f"no level-symmetric set for S{N}")
    mu1 = _LQN_MU1[N]
    h = N // 2
    if N == 2:
        cos = np.array([mu1])
    else:
        delta = 2.0 * (1.0 - 3.0 * mu1 * mu1) / (N - 2)
        cos = np.sqrt(mu1 * mu1 + delta * np.arange(h))
    trip = []
    cls = []
    for i in range(1, h + 1):
        for j in range(1, h + 1):
            k = h + 2 - i - j
            if 1 <= k <= h:
                v = np.array([cos[i - 1], cos[j - 1], cos[k - 1]])
                trip.append(v / np.linalg.norm(v))
                cls.append(tuple(sorted((i, j, k))))
    trip = np.array(trip)
    keys = sorted(set(cls))
    member = np.array([[1.0 if c == key else 0.0 for key in keys] for c in cls])
    moments = np.array([[(trip[member[:, q] > 0, 0] ** (2 * m)).sum() for q in range(len(keys))]
                        for m in range(h)])
    target = 1.0 / (2.0 * np.arange(h) + 1.0)
    wc = np.linalg.lstsq(moments, target, rcond=None)[0]
    w_oct = member @ wc                     # per point, octant sum 1
    per = trip.shape[0]
    L = 8 * per
    mu = np.empty(L)
    eta = np.empty(L)
    xi = np.empty(L)
    w = np.empty(L)
    for o in range(8):
        sx = 1.0 if (o & 1) else -1.0
        sy = 1.0 if (o & 2) else -1.0
        sz = 1.0 if (o & 4) else -1.0
        sl = slice(o * per, (o + 1) * per)
        mu[sl] = sx * trip[:, 0]
        eta[sl] = sy * trip[:, 1]
        xi[sl] = sz * trip[:, 2]
        w[sl] = w_oct / 8.0
    return Quadrature(mu, eta, xi, w)


def _draw_materials(rng, n_mat: int, G: int, upscatter_groups: int = 0):
    """Cross sections of ``n_mat`` materials as in the 32^3 four-group case."""
    sigma_t = rng.uniform(0.5, 2.0, size=(n_mat, G))
    sigma_s = np.zeros((n_mat, G, G))
    for m in range(n_mat):
        for gp in range(G):
            for g in range(gp, G):
                sigma_s[m, g, gp] = rng.uniform(0.0, 0.3) * sigma_t[m, gp]
        if upscatter_groups:
            lo = G - upscatter_groups
            for gp in range(lo, G):
                for g in range(lo, gp):
                    sigma_s[m, g, gp] = rng.uniform(0.0, 0.05) * sigma_t[m, gp]
        for gp in range(G):
            s = sigma_s[m, :, gp].sum()
            cap = 0.9 * sigma_t[m, gp]
            if s > cap:
                sigma_s[m, :, gp] *= cap / s
    nu_sigma_f = rng.uniform(0.0, 0.2, size=(n_mat, G))
    chi = rng.uniform(0.0, 1.0, size=G)
    chi /= chi.sum()
    return sigma_t, sigma_s, nu_sigma_f, chi


def _psi0(rng, G: int, L: int, l: int):
    e = rng.uniform(0.5, 1.5, size=G) if G > 1 else np.ones(1)
    a = rng.uniform(0.5, 1.5, size=L)
    bits = rng.uniform(0.5, 1.5, size=(3, l, 2))
    return e, a, bits


def homogeneous(l: int = 3, N: int = 2, seed: int = 0, rmax: int = 8,
                tol: float = 1e-10, tol_k: float = 1e-8,
                sigma_t: float = 1.0, sigma_s: float = 0.5,
                nu_sigma_f: float = 0.6, jitter: float = 0.1,
                boundary: str = "vacuum", name: Optional[str] = None) -> Workload:
    """One-group homogeneous cube (the 8^3 S2 smallest case by default)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(-1.0, 1.0, size=3) * jitter
    st = sigma_t * (1 + u[0])
    ss = sigma_s * (1 + u[1])
    nf = nu_sigma_f * (1 + u[2])
    quad = level_symmetric(N)
    e, a, bits = _psi0(rng, 1, quad.L, l)
    return Workload(
        name=name or f"homogeneous_n{1 << l}_S{N}", l=l, G=1, quad=quad,
        cuts=[[], [], []], block_mat=np.zeros((1, 1, 1), dtype=np.int64),
        sigma_t=np.array([[st]]), sigma_s=np.array([[[ss]]]),
        nu_sigma_f=np.array([[nf]]), chi=np.ones(1),
        psi0_energy=e, psi0_angle=a, psi0_bits=bits,
        rmax=rmax, tol=tol, tol_k=tol_k, seed=seed, boundary=boundary)


def inner_box(l: int = 5, G: int = 4, N: int = 4, seed: int = 1, rmax: int = 32,
              tol: float = 1e-8, tol_k: float = 1e-8,
              name: Optional[str] = None) -> Workload:
    """Two-region cube: a seeded random inner box in an outer material."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 1 << l
    M = n - 1
    cuts = []
    for _ in range(3):
        a, b = sorted(rng.choice(np.arange(1, M), size=2, replace=False).tolist())
        cuts.append([a + 1, b + 1])      # blocks: cells 1..a, a+1..b, b+1..M
    block_mat = np.zeros((3, 3, 3), dtype=np.int64)
    block_mat[1, 1, 1] = 1
    st, ss, nf, chi = _draw_materials(rng, 2, G)
    quad = level_symmetric(N)
    e, a_, bits = _psi0(rng, G, quad.L, l)
    return Workload(
        name=name or f"inner_box_n{n}_G{G}_S{N}", l=l, G=G, quad=quad, cuts=cuts,
        block_mat=block_mat, sigma_t=st, sigma_s=ss, nu_sigma_f=nf, chi=chi,
        psi0_energy=e, psi0_angle=a_, psi0_bits=bits, rmax=rmax, tol=tol,
        tol_k=tol_k, seed=seed)


def checkerboard(l: int = 7, G: int = 8, N: int = 8, blocks: int = 4,
                 n_mat: int = 4, seed: int = 2, rmax: int = 64,
                 tol: float = 1e-8, tol_k: float = 1e-8,
                 upscatter_groups: int = 0, permutation: bool = False,
                 name: Optional[str] = None) -> Workload:
    """``blocks^3`` node-aligned blocks, each drawn from ``n_mat`` materials."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 1 << l
    step = n // blocks
    cuts = [[b * step + 1 for b in range(1, blocks)] for _ in range(3)]
    if permutation:
        block_mat = rng.permutation(blocks ** 3).reshape(blocks, blocks, blocks)
        n_mat = blocks ** 3
    else:
        block_mat = rng.integers(0, n_mat, size=(blocks, blocks, blocks))
    st, ss, nf, chi = _draw_materials(rng, n_mat, G, upscatter_groups)
    quad = level_symmetric(N)
    e, a, bits = _psi0(rng, G, quad.L, l)
    return Workload(
        name=name or f"checkerboard_n{n}_G{G}_S{N}", l=l, G=G, quad=quad,
        cuts=cuts, block_mat=block_mat.astype(np.int64), sigma_t=st,
        sigma_s=ss, nu_sigma_f=nf, chi=chi, psi0_energy=e, psi0_angle=a,
        psi0_bits=bits, rmax=rmax, tol=tol, tol_k=tol_k, seed=seed)


def gauss_legendre_slab(N: int) -> Quadrature:
    """Ordinates for a slab along x: the N-point Gauss-Legendre cosines mu
    (weights normalized to 1/8 per octant), with eta = xi = sqrt((1 - mu^2)/2)
    so that each direction is a unit vector; the y and z cosines do not enter
    a solution that is uniform in y and z."""
    mu_gl, w_gl = np.polynomial.legendre.leggauss(N)
    pos = mu_gl > 0
    mu_m, w_m = mu_gl[pos], w_gl[pos] / w_gl[pos].sum()
    per = mu_m.size
    tr = np.sqrt((1.0 - mu_m ** 2) / 2.0)
    L = 8 * per
    mu, eta, xi, w = (np.empty(L) for _ in range(4))
    for o in range(8):
        sl = slice(o * per, (o + 1) * per)
        mu[sl] = (1.0 if o & 1 else -1.0) * mu_m
        eta[sl] = (1.0 if o & 2 else -1.0) * tr
        xi[sl] = (1.0 if o & 4 else -1.0) * tr
        w[sl] = w_m / 8.0
    return Quadrature(mu, eta, xi, w)


def slab(N: int, lx: int, sigma_t: float, sigma_s: float, nu_sigma_f: float, width: float,
         seed: int = 0, rmax: int = 32, tol: float = 1e-10, tol_k: float = 1e-10,
         name: Optional[str] = None) -> Workload:
    """One-group homogeneous slab of the given width along x (vacuum faces),
    2^lx nodes across it; y and z have two nodes and periodic faces, so the
    solution is uniform in y and z (a one-dimensional slab)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    quad = gauss_legendre_slab(N)
    a = rng.uniform(0.5, 1.5, size=quad.L)
    bits = np.ones((3, lx, 2))
    bits[2] = rng.uniform(0.5, 1.5, size=(lx, 2))
    return Workload(
        name=name or f"slab_nx{1 << lx}_S{N}", l=lx, G=1, quad=quad,
        cuts=[[], [], []], block_mat=np.zeros((1, 1, 1), dtype=np.int64),
        sigma_t=np.array([[sigma_t]]), sigma_s=np.array([[[sigma_s]]]),
        nu_sigma_f=np.array([[nu_sigma_f]]), chi=np.ones(1),
        psi0_energy=np.ones(1), psi0_angle=a, psi0_bits=bits, rmax=rmax, tol=tol,
        tol_k=tol_k, seed=seed, periodic=(True, True, False), l_axes=(1, 1, lx),
        lengths=(1.0, 1.0, float(width)))


def config(idx: int, **over) -> Workload:
    """The five named workloads of this project, by index.

    0: 8^3 nodes, 1 group, S2, homogeneous jittered, rank cap 8, tol 1e-10.
    1: 32^3 nodes, 4 groups, S4, two-region, rank cap 32, tol 1e-8.
    2: 128^3 nodes, 8 groups, S8, 4x4x4 checkerboard of 4 materials, cap 64.
    4: 1024^3 nodes, 16 groups, S16, 2x2x2 permutation of 8 materials,
       upscatter among the lowest 4 groups, cap 96.
    (3 is the batch of ``batch_instances``.)
    """
    if idx == 0:
        return homogeneous(**over)
    if idx == 1:
        return inner_box(**over)
    if idx == 2:
        return checkerboard(**over)
    if idx == 4:
        kw = dict(l=10, G=16, N=16, blocks=2, seed=4, rmax=96, tol=1e-7,
                  tol_k=1e-6, upscatter_groups=4, permutation=True)
        kw.update(over)
        return checkerboard(**kw)
    raise ValueError(f"no single workload {idx}")


def batch_instances(count: int = 256, base_seed: int = 1000) -> List[Workload]:
    """Independent uneven instances: n in {16,32,64}, G 1..8, S2..S8, cap 4..48."""
    out = []
    for j in range(count):
        rng = np.random.Generator(np.random.PCG64(base_seed + j))
        l = int(rng.integers(4, 7))
        G = int(rng.integers(1, 9))
        N = int(rng.choice([2, 4, 6, 8]))
        rmax = int(rng.integers(4, 49))
        w = inner_box(l=l, G=G, N=N, seed=base_seed + j, rmax=rmax, tol=1e-6,
                      tol_k=1e-6, name=f"batch{j}")
        out.append(w)
    return out
