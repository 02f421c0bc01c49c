"""ctypes driver for the C transport-sweep checker (``dd_sweep.c``).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Pins (tests/test_oracle_sweep.py):
  * reflective homogeneous cube: k -> nu_sigma_f/(sigma_t - sigma_s) (one
    group) or nu_sigma_f^T (diag sigma_t - Sigma_s)^{-1} chi (many groups);
    the reflection here is lagged (incoming faces from the previous iterate),
    so only the limit is the closed form; its limit equals the eigenvalue of
    the dense operator with mirror rows (tests/test_oracle_pins.py);
  * one power step equals H^{-1}(S + F/k) psi by a sparse LU of the dense
    equation-row operator, with k from sum(F psi) of the dense F; the
    fission functional equals sum(F psi) for all three dense assemblies;
    the source equals the cell rows of (S + F/k) psi;
  * the sweep equals a dense LU solve of the equation-row operator;
  * the converged k equals the brute-force generalized eigenvalue;
  * neutron balance: leakage + absorption = in-scatter + production / k;
  * inflow faces are exactly zero; the scalar flux is mirror-symmetric in a
    homogeneous cube.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dd_sweep.c")
_LIB = os.path.join(_HERE, "libddsweep.so")


def build(force: bool = False) -> str:
    """Compile the checker with gcc (plain C, OpenMP over (group, direction)).

    -march=x86-64-v3 (AVX2, FMA) rather than native, so that the library
    built on one host also runs on any other recent x86-64 host."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("G", ctypes.c_int64), ("L", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("ny", ctypes.c_int64), ("nx", ctypes.c_int64),
                ("hz", ctypes.c_double), ("hy", ctypes.c_double), ("hx", ctypes.c_double),
                ("mu", ctypes.c_void_p), ("eta", ctypes.c_void_p), ("xi", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("mat", ctypes.c_void_p), ("sigma_t", ctypes.c_void_p),
                ("sigma_s", ctypes.c_void_p), ("nu_sigma_f", ctypes.c_void_p),
                ("chi", ctypes.c_void_p), ("reflective", ctypes.c_int64 * 3)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.POINTER(_Problem)
        d = ctypes.c_void_p
        _lib.dd_phi8.argtypes = [P, d, d]
        _lib.dd_source.argtypes = [P, d, ctypes.c_double, d]
        _lib.dd_fission_total.argtypes = [P, d]
        _lib.dd_fission_total.restype = ctypes.c_double
        _lib.dd_sweep.argtypes = [P, d, d, d]
        _lib.dd_power_iteration.argtypes = [P, d, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int64, d]
        _lib.dd_power_iteration.restype = ctypes.c_int64
        _lib.dd_power_step.argtypes = [P, d, ctypes.c_double, d]
        _lib.dd_power_step.restype = ctypes.c_double
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Problem:
    """Dense-grid description of one instance for the C checker.

    Holds its own contiguous copies of every array so the C side can keep
    raw pointers for the lifetime of this object.
    """

    def __init__(self, G, mu, eta, xi, w, mat, sigma_t, sigma_s, nu_sigma_f, chi,
                 shape: Tuple[int, int, int], spacing: Tuple[float, float, float],
                 reflective=(False, False, False)):
        self.G = int(G)
        self.shape = tuple(int(s) for s in shape)
        self.L = int(len(mu))
        self._arrays = dict(
            mu=np.ascontiguousarray(mu, dtype=np.float64),
            eta=np.ascontiguousarray(eta, dtype=np.float64),
            xi=np.ascontiguousarray(xi, dtype=np.float64),
            w=np.ascontiguousarray(w, dtype=np.float64),
            mat=np.ascontiguousarray(mat, dtype=np.int64).reshape(-1),
            sigma_t=np.ascontiguousarray(sigma_t, dtype=np.float64),
            sigma_s=np.ascontiguousarray(sigma_s, dtype=np.float64),
            nu_sigma_f=np.ascontiguousarray(nu_sigma_f, dtype=np.float64),
            chi=np.ascontiguousarray(chi, dtype=np.float64))
        nz, ny, nx = self.shape
        assert self._arrays["mat"].size == (nz - 1) * (ny - 1) * (nx - 1)
        assert self.L % 8 == 0
        a = self._arrays
        self._s = _Problem(self.G, self.L, nz, ny, nx, spacing[0], spacing[1], spacing[2],
                           _ptr(a["mu"]).value, _ptr(a["eta"]).value, _ptr(a["xi"]).value,
                           _ptr(a["w"]).value, _ptr(a["mat"]).value, _ptr(a["sigma_t"]).value,
                           _ptr(a["sigma_s"]).value, _ptr(a["nu_sigma_f"]).value,
                           _ptr(a["chi"]).value,
                           (ctypes.c_int64 * 3)(*[int(bool(r)) for r in reflective]))

    @classmethod
    def from_workload(cls, wl, reflective=None):
        shape = tuple(wl.axis_nodes(ax) for ax in range(3))
        spacing = tuple(wl.axis_spacing(ax) for ax in range(3))
        if reflective is None:
            reflective = (wl.boundary == "reflective",) * 3
        q = wl.quad
        return cls(wl.G, q.mu, q.eta, q.xi, q.w, wl.cell_material(), wl.sigma_t,
                   wl.sigma_s, wl.nu_sigma_f, wl.chi, shape, spacing, reflective)

    @property
    def n_unknowns(self) -> int:
        nz, ny, nx = self.shape
        return self.G * self.L * nz * ny * nx

    @property
    def n_cells(self) -> int:
        nz, ny, nx = self.shape
        return (nz - 1) * (ny - 1) * (nx - 1)

    def _psi(self, psi):
        psi = np.ascontiguousarray(psi, dtype=np.float64).reshape(-1)
        assert psi.size == self.n_unknowns
        return psi

    def phi8(self, psi) -> np.ndarray:
        psi = self._psi(psi)
        out = np.empty(self.G * self.n_cells)
        _load().dd_phi8(ctypes.byref(self._s), _ptr(psi), _ptr(out))
        return out

    def source(self, psi, k: float) -> np.ndarray:
        phi = self.phi8(psi)
        q = np.empty_like(phi)
        _load().dd_source(ctypes.byref(self._s), _ptr(phi), 1.0 / k, _ptr(q))
        return q

    def fission_total(self, psi) -> float:
        return float(_load().dd_fission_total(ctypes.byref(self._s), _ptr(self.phi8(psi))))

    def sweep(self, q, psi_prev=None) -> np.ndarray:
        q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
        assert q.size == self.G * self.n_cells
        prev = np.zeros(self.n_unknowns) if psi_prev is None else self._psi(psi_prev)
        out = np.empty(self.n_unknowns)
        _load().dd_sweep(ctypes.byref(self._s), _ptr(q), _ptr(prev), _ptr(out))
        return out

    def power_step(self, psi, k: float):
        """One step of eq. k_eff_fixed_points; returns (unnormalized psi_next, k_next)."""
        psi = self._psi(psi)
        out = np.empty(self.n_unknowns)
        kn = _load().dd_power_step(ctypes.byref(self._s), _ptr(psi), float(k), _ptr(out))
        return out, float(kn)

    def power_iteration(self, psi0, k0: float = 1.0, tol_k: float = 1e-8,
                        max_steps: int = 1000):
        """Returns (k history [steps+1], final unit-norm psi)."""
        psi = self._psi(psi0).copy()
        hist = np.empty(max_steps + 1)
        steps = _load().dd_power_iteration(ctypes.byref(self._s), _ptr(psi), float(k0),
                                           float(tol_k), int(max_steps), _ptr(hist))
        return hist[:steps + 1].copy(), psi


def dense_psi0(wl) -> np.ndarray:
    """Dense initial flux: outer product of the seeded rank-1 factors."""
    axes = []
    for ax in range(3):
        v = np.ones(1)
        for b in range(wl.axis_bits(ax)):
            v = np.kron(v, wl.psi0_bits[ax, b])
        axes.append(v)
    e = wl.psi0_energy if wl.G > 1 else np.ones(1)
    out = np.einsum("g,a,k,j,i->gakji", e, wl.psi0_angle, axes[0], axes[1], axes[2])
    return out.reshape(-1)


def run_workload(wl, max_steps: int = 1000, psi0: Optional[np.ndarray] = None,
                 reflective=None):
    """Exact discrete power iteration of one workload from its seeded start."""
    prob = Problem.from_workload(wl, reflective)
    start = dense_psi0(wl) if psi0 is None else psi0
    return prob.power_iteration(start, 1.0, wl.tol_k, max_steps)
