"""tt_power_step_async: the fixed-rank power step with no host
synchronization (eq. TT_k_eff_fixed_points with one-site alternating sweeps
at psi's settled ranks), checked against the checker's exact step from the
same iterate, and recorded by a stream capture whose replays repeat the
eagerly enqueued step bit for bit.
"""
import numpy as np
import pytest

from oracle import sweep, tt as OT
from paper_2309_03347_amd import workload as W

pytestmark = pytest.mark.gpu


def _unit(v):
    v = v / np.linalg.norm(v)
    return v if v.sum() >= 0 else -v


def _settled(wl, **kw):
    # rank cap lifted so the tolerance sets the ranks (the adaptive steps reach
    # them; the fixed-rank steps then need no more)
    from paper_2309_03347_amd.solver import KeffSolver
    s = KeffSolver(wl, rmax=256, max_sweeps=12, **kw)
    for _ in range(3):
        s.step()
    return s


@pytest.mark.parametrize("maker", [
    lambda: W.inner_box(l=3, G=2, N=4, seed=21, rmax=64, tol=1e-10),
    lambda: W.homogeneous(l=3, N=2, seed=3, tol=1e-10),
])
def test_async_steps_match_oracle(cuda, maker):
    import torch
    from paper_2309_03347_amd import native
    wl = maker()
    s = _settled(wl)
    prob = sweep.Problem.from_workload(wl)
    psi = OT.full_vec(s.psi_cores())
    k = s.history[-1].k
    buf = native.step_info_buffer()
    for step in range(3):
        print(f"async step {step}", flush=True)
        s.native.step_async(buf)
        torch.cuda.synchronize()
        info = native.read_step_info(buf)
        ref, kref = prob.power_step(psi, k)
        got = OT.full_vec(s.psi_cores())
        assert info["status"] in (native.TT_OK, native.TT_E_NOCONV), info
        assert abs(info["k_prev"] - k) <= 1e-14 * abs(k)
        assert abs(info["k"] - kref) <= 1e-8 * abs(kref), (step, info["k"], kref)
        assert np.linalg.norm(_unit(got) - _unit(ref)) <= 1e-6, step
        assert abs(np.linalg.norm(got) - 1.0) <= 1e-12
        psi, k = got, info["k"]
    # a regular step after asynchronous ones still matches the checker
    rec = s.step()
    ref, kref = prob.power_step(psi, k)
    assert abs(rec.k - kref) <= 1e-8 * abs(kref)
    s.close()


def test_captured_async_step_replays_match_eager_steps(cuda):
    # one solver steps eagerly, its twin (same operators, same adaptive
    # history, so the same state) replays a captured step; between replays
    # the program does its own work and synchronizes.  Every replay must equal
    # the eager step bit for bit.
    import torch
    from paper_2309_03347_amd import native
    wl = W.inner_box(l=3, G=2, N=4, seed=21, rmax=64, tol=1e-10)
    a = _settled(wl)
    b = _settled(wl)
    for ca, cb in zip(a.psi_cores(), b.psi_cores()):
        assert np.array_equal(ca, cb)
    buf_a, buf_b = native.step_info_buffer(), native.step_info_buffer()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    print("capturing one asynchronous step", flush=True)
    with torch.cuda.graph(g):
        b.native.step_async(buf_b, sweeps=3)
    torch.cuda.synchronize()
    for r in range(3):
        print(f"replay {r}", flush=True)
        a.native.step_async(buf_a, sweeps=3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        x = torch.randn(1 << 16, device="cuda")     # eager work between replays
        (x * x).sum().item()
        ia, ib = native.read_step_info(buf_a), native.read_step_info(buf_b)
        assert ia == ib, (r, ia, ib)
        for ca, cb in zip(a.psi_cores(), b.psi_cores()):
            assert np.array_equal(ca, cb), r
    a.close()
    b.close()


def test_capped_graphs_replay_concurrently_on_two_streams(cuda):
    # two instances' fixed-rank steps captured with their persistent grids
    # capped at 128 workgroups and replayed at once on two streams equal the
    # same steps enqueued eagerly one after the other
    import torch
    from paper_2309_03347_amd import native
    wls = [W.inner_box(l=3, G=2, N=4, seed=21, rmax=64, tol=1e-10),
           W.homogeneous(l=3, N=2, seed=3, tol=1e-10)]
    eager = [_settled(w) for w in wls]
    graphed = [_settled(w) for w in wls]
    bufs_e = [native.step_info_buffer() for _ in wls]
    bufs_g = [native.step_info_buffer() for _ in wls]
    graphs = []
    torch.cuda.synchronize()
    native.set_grid_cap(128)
    try:
        for s, b in zip(graphed, bufs_g):
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                s.native.step_async(b, sweeps=3)
            graphs.append(g)
    finally:
        native.set_grid_cap(0)
    streams = [torch.cuda.Stream() for _ in wls]
    for r in range(2):
        print(f"concurrent replay {r}", flush=True)
        # the same cap, so both take the same work split (and sum order)
        native.set_grid_cap(128)
        try:
            for s, b in zip(eager, bufs_e):
                s.native.step_async(b, sweeps=3)
        finally:
            native.set_grid_cap(0)
        torch.cuda.synchronize()
        for g, st in zip(graphs, streams):
            with torch.cuda.stream(st):
                g.replay()
        torch.cuda.synchronize()
        for i in range(len(wls)):
            assert native.read_step_info(bufs_e[i]) == native.read_step_info(bufs_g[i]), (r, i)
            for ca, cb in zip(eager[i].psi_cores(), graphed[i].psi_cores()):
                assert np.array_equal(ca, cb), (r, i)
    for s in eager + graphed:
        s.close()


def test_one_graph_forks_instances_over_streams(cuda):
    # three instances' fixed-rank steps captured into ONE graph: the capture
    # stream forks to two side streams, each instance's step is recorded on
    # one of them, and both join back before the capture ends; replaying the
    # graph equals the same steps enqueued eagerly under the same grid cap
    import torch
    from paper_2309_03347_amd import native
    wls = [W.inner_box(l=3, G=2, N=4, seed=21, rmax=64, tol=1e-10),
           W.homogeneous(l=3, N=2, seed=3, tol=1e-10),
           W.homogeneous(l=2, N=4, seed=5, tol=1e-10)]
    eager = [_settled(w) for w in wls]
    graphed = [_settled(w) for w in wls]
    bufs_e = [native.step_info_buffer() for _ in wls]
    bufs_g = [native.step_info_buffer() for _ in wls]
    side = [torch.cuda.Stream() for _ in range(2)]
    cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    native.set_grid_cap(128)
    try:
        with torch.cuda.graph(g, stream=cap):
            for st in side:
                st.wait_stream(cap)
            for i, (s, b) in enumerate(zip(graphed, bufs_g)):
                with torch.cuda.stream(side[i % 2]):
                    s.native.step_async(b, sweeps=3)
            for st in side:
                cap.wait_stream(st)
    finally:
        native.set_grid_cap(0)
    for r in range(2):
        print(f"one-graph replay {r}", flush=True)
        native.set_grid_cap(128)
        try:
            for s, b in zip(eager, bufs_e):
                s.native.step_async(b, sweeps=3)
        finally:
            native.set_grid_cap(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(len(wls)):
            assert native.read_step_info(bufs_e[i]) == native.read_step_info(bufs_g[i]), (r, i)
            for ca, cb in zip(eager[i].psi_cores(), graphed[i].psi_cores()):
                assert np.array_equal(ca, cb), (r, i)
    for s in eager + graphed:
        s.close()
