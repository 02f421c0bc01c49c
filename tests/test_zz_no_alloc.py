"""tt_local_solve_noalloc (static scratch, no workspace) against tt_local_solve.

Two calls in a row share the library's static scratch; the second uses a
smaller system, so leftovers of the first must not leak into it.  Each result
is checked against the workspace entry point's on the same inputs and against
the checker's local operator (relative residual).
"""
import numpy as np
import pytest

from oracle import tt as OT

pytestmark = pytest.mark.gpu


def _system(rng, ra, RL, n, RR, rc, diag=True):
    phiL = rng.standard_normal((ra, RL, ra)) / np.sqrt(ra * RL)
    phiR = rng.standard_normal((rc, RR, rc)) / np.sqrt(rc * RR)
    A = rng.standard_normal((RL, n, n, RR)) / np.sqrt(n * RL * RR)
    phiL[:, 0, :] += 8.0 * np.eye(ra)
    phiR[:, 0, :] += np.eye(rc)
    A[0, :, :, 0] += np.eye(n)
    if n > 2 and diag:
        A = np.einsum("bijc,ij->bijc", A, np.eye(n))
    f = rng.standard_normal(ra * n * rc)
    return phiL, A, phiR, f


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("method,big,small", [
    (2, (36, 8, 2, 8, 36), (12, 4, 2, 6, 10)),     # persistent GMRES
    (1, (6, 4, 3, 4, 7), (3, 3, 2, 2, 4)),         # dense Gauss-Jordan
    (3, (6, 4, 24, 4, 6), (4, 3, 8, 3, 5)),        # mode-diagonal blocks
])
def test_noalloc_matches_workspace_entry_point(cuda, method, big, small):
    from paper_2309_03347_amd import native
    rng = np.random.default_rng(100 + method)
    for dims in (big, small):
        ra, RL, n, RR, rc = dims
        phiL, A, phiR, f = _system(rng, ra, RL, n, RR, rc)
        shape = (ra, n, rc)
        args = (_t(phiL), _t(A), _t(phiR), _t(f.reshape(shape)), _t(np.zeros(shape)))
        kw = dict(method=method, tol=1e-12, max_iter=2000, restart=60, direct_max=0)
        print(f"noalloc method={method} dims={dims}", flush=True)
        x_ref, info_ref = native.tt_local_solve(*args, **kw)
        x, info = native.tt_local_solve_noalloc(*args, **kw)
        x, x_ref = x.cpu().numpy().reshape(-1), x_ref.cpu().numpy().reshape(-1)
        assert info["method"] == info_ref["method"] == method
        assert info["converged"] and info_ref["converged"]
        assert np.linalg.norm(x - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
        if method == 3:
            # only the mode-diagonal entries enter the block solve
            Ad = np.einsum("bijc,ij->bijc", A, np.eye(n))
            r = OT.local_apply(phiL, Ad, phiR, x) - f
        else:
            r = OT.local_apply(phiL, A, phiR, x) - f
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(f)
