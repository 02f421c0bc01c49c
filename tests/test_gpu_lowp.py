"""BF16 and FP16 matrix-core contractions and the refined mixed-precision solves.

tt_local_apply applies the projected local operator of the alternating solve
(Section 3.3) as three contractions; in precision 2 they run on the BF16
matrix cores (operands rounded to BF16, FP32 accumulation).  Its result is
held to the rounding bound of that arithmetic: each product a b of two
BF16-rounded operands has relative error below 2 * 2^-9 + 2^-18, so each
contraction stage is off by at most that factor of the same contraction of
absolute values, plus the FP32 accumulation (K 2^-24).  Over the three stages
and the rounding of the two intermediates the bound used is
    |y - y_ref| <= 2e-2 * (|PhiL| (x) |A| (x) |PhiR|) |x|,
with y_ref and the absolute product from the checker.

In precision 3 the contractions run on the FP16 matrix cores.  Every row of the
left operand and column of the right operand of each contraction is divided,
per 32-deep block of the contracted index, by the power of two just above its
largest magnitude before the cast, and the block's FP32 partial product is
multiplied back by both scales.  A product of two scaled entries then has
relative error below 2 * 2^-11 + 2^-22; an entry smaller than 2^-14 of its
block's largest falls below FP16's normal range and is off by at most 2^-25 of
the block scale.  Per contraction stage that gives 2^-10 + K 2^-24 (K <= 4,216
here: 2.5e-4) of the contraction of absolute values, three stages 3.7e-3, and
the bound used is
    |y - y_ref| <= 5e-3 * (|PhiL| (x) |A| (x) |PhiR|) |x| + 1e-6 max(...),
the second term covering the subnormal entries, which for these Gaussian
operands stay below 1e-6 of the largest absolute product.

The mixed solves (precisions 2 and 3) use those products inside each GMRES
restart cycle and the FP64 residual at every restart, so they are held to the
FP64 bar.
"""
import numpy as np
import pytest

from oracle import sweep, tt as OT
from paper_2309_03347_amd import workload as W

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _system(rng, ra, RL, n, RR, rc):
    phiL = rng.standard_normal((ra, RL, ra)) / np.sqrt(ra * RL)
    phiR = rng.standard_normal((rc, RR, rc)) / np.sqrt(rc * RR)
    A = rng.standard_normal((RL, n, n, RR)) / np.sqrt(n * RL * RR)
    phiL[:, 0, :] += 8.0 * np.eye(ra)
    phiR[:, 0, :] += np.eye(rc)
    A[0, :, :, 0] += np.eye(n)
    f = rng.standard_normal(ra * n * rc)
    return phiL, A, phiR, f


SHAPES = [
    # ra, RL, n, RR, rc: tile edges of the 64 x 64 output tiles and 32-deep k-steps
    (6, 4, 2, 5, 7),
    (40, 8, 2, 8, 40),
    (20, 6, 3, 66, 70),
    (68, 60, 2, 62, 68),      # the rank-64 spatial cores of the 128^3 workload
    (1, 1, 2, 1, 1),
]


@pytest.mark.parametrize("ra,RL,n,RR,rc", SHAPES)
def test_local_apply_fp64_and_bf16(cuda, ra, RL, n, RR, rc):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(ra * 7 + rc)
    phiL, A, phiR, _ = _system(rng, ra, RL, n, RR, rc)
    x = rng.standard_normal(ra * n * rc)
    ref = OT.local_apply(phiL, A, phiR, x)
    absref = OT.local_apply(np.abs(phiL), np.abs(A), np.abs(phiR), np.abs(x))
    y64 = native.tt_local_apply(_t(phiL), _t(A), _t(phiR), _t(x.reshape(ra, n, rc)), 0)
    y64 = y64.cpu().numpy().reshape(-1)
    assert np.abs(y64 - ref).max() <= 1e-13 * absref.max()
    ylp = native.tt_local_apply(_t(phiL), _t(A), _t(phiR), _t(x.reshape(ra, n, rc)), 2)
    ylp = ylp.cpu().numpy().reshape(-1)
    err = np.abs(ylp - ref)
    assert np.all(err <= 2e-2 * absref + 1e-300), (err / absref).max()
    if ra * rc > 1:
        # the products really ran in BF16: some entry is off by more than FP32 rounding
        assert (err / absref).max() > 1e-6


@pytest.mark.parametrize("ra,RL,n,RR,rc", SHAPES)
def test_local_apply_fp16_block_scaled(cuda, ra, RL, n, RR, rc):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(ra * 11 + rc)
    phiL, A, phiR, _ = _system(rng, ra, RL, n, RR, rc)
    x = rng.standard_normal(ra * n * rc)
    ref = OT.local_apply(phiL, A, phiR, x)
    absref = OT.local_apply(np.abs(phiL), np.abs(A), np.abs(phiR), np.abs(x))
    args = (_t(phiL), _t(A), _t(phiR), _t(x.reshape(ra, n, rc)))
    y16 = native.tt_local_apply(*args, 3).cpu().numpy().reshape(-1)
    err16 = np.abs(y16 - ref)
    assert np.all(err16 <= 5e-3 * absref + 1e-6 * absref.max()), (err16 / absref).max()
    if ra * rc > 1:
        ybf = native.tt_local_apply(*args, 2).cpu().numpy().reshape(-1)
        rel16 = (err16 / absref).max()
        # reduced precision really ran, and with three more mantissa bits than BF16
        assert rel16 > 1e-7
        assert rel16 < (np.abs(ybf - ref) / absref).max()


def test_local_apply_fp16_scales_each_row_and_column(cuda):
    # Entries far outside FP16's range (2^-24 .. 65504), and rows of PhiL and
    # PhiR whose magnitudes differ by 1e16: one scale per core would send the
    # small rows below FP16's range (or the large ones above it); the per-row,
    # per-column block scales keep every output entry to the relative bound.
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(77)
    ra, RL, n, RR, rc = 20, 6, 3, 10, 24
    phiL, A, phiR, _ = _system(rng, ra, RL, n, RR, rc)
    phiL = phiL * np.logspace(-8, 8, ra)[:, None, None] * 1e9
    phiR = phiR * np.logspace(6, -10, rc)[:, None, None]
    A = A * 1e-7
    x = rng.standard_normal(ra * n * rc) * 3e5
    ref = OT.local_apply(phiL, A, phiR, x)
    absref = OT.local_apply(np.abs(phiL), np.abs(A), np.abs(phiR), np.abs(x))
    y16 = native.tt_local_apply(_t(phiL), _t(A), _t(phiR), _t(x.reshape(ra, n, rc)), 3)
    y16 = y16.cpu().numpy().reshape(-1)
    assert np.all(np.isfinite(y16))
    rel = np.abs(y16 - ref) / absref
    assert rel.max() <= 5e-3, rel.max()


@pytest.mark.parametrize("precision", [2, 3])
@pytest.mark.parametrize("ra,RL,n,RR,rc,restart", [
    (12, 6, 2, 6, 10, 40),
    (36, 56, 2, 56, 36, 60),
    (9, 5, 3, 4, 11, 12),
])
def test_refined_lowp_local_solve_meets_fp64_tolerance(cuda, ra, RL, n, RR, rc, restart,
                                                       precision):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(3 * ra + rc)
    phiL, A, phiR, f = _system(rng, ra, RL, n, RR, rc)
    shape = (ra, n, rc)
    args = (_t(phiL), _t(A), _t(phiR), _t(f.reshape(shape)), _t(np.zeros(shape)))
    x, info = native.tt_local_solve(*args, method=4, tol=1e-12, max_iter=4000,
                                    restart=restart, direct_max=0, precision=precision)
    assert info["converged"] and info["rel_res"] <= 1e-11, info
    r = OT.local_apply(phiL, A, phiR, x.cpu().numpy().reshape(-1)) - f
    assert np.linalg.norm(r) <= 1e-11 * np.linalg.norm(f)
    x64, info64 = native.tt_local_solve(*args, method=4, tol=1e-12, max_iter=4000,
                                        restart=restart, direct_max=0, precision=0)
    assert np.linalg.norm(x.cpu().numpy() - x64.cpu().numpy()) <= 1e-10 * np.linalg.norm(
        x64.cpu().numpy())


def _unit(v):
    v = v / np.linalg.norm(v)
    return v if v.sum() >= 0 else -v


@pytest.mark.parametrize("precision", [2, 3])
def test_power_steps_lowp_mode_match_oracle(cuda, precision):
    # every local GMRES solve on the multi-launch path with BF16 (2) or
    # block-scaled FP16 (3) products in its cycles; the refined solves
    # converge in FP64, so the FP64 bar holds
    from paper_2309_03347_amd.solver import KeffSolver
    wl = W.inner_box(l=3, G=2, N=4, seed=21, rmax=64, tol=1e-10)
    s = KeffSolver(wl, rmax=256, kick=8, max_sweeps=60, precision=precision, krylov_path=1)
    s64 = KeffSolver(wl, rmax=256, kick=8, max_sweeps=60, precision=0, ops=s.ops)
    prob = sweep.Problem.from_workload(wl)
    psi = OT.full_vec(s.native.psi().cores())
    k = 1.0
    for step in range(3):
        print(f"precision {precision} mode step {step}", flush=True)
        rec = s.step()
        rec64 = s64.step()
        ref, kref = prob.power_step(psi, k)
        got = OT.full_vec(s.psi_cores())
        assert abs(rec.k - kref) <= 1e-8 * abs(kref), (step, rec.k, kref)
        assert np.linalg.norm(_unit(got) - _unit(ref)) <= 1e-6, step
        # mixed against the FP64 twin: the 1e-5 bar of the mixed mode, met by far
        assert abs(rec.k - rec64.k) <= 1e-5 * abs(rec64.k)
        psi, k = got, rec.k
    s.close()
    s64.close()
