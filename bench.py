"""Benchmark: TT/QTT power-iteration steps per second on one MI355X.

Workload (default): 128^3 nodes, 8 energy groups, S8 level-symmetric
(80 directions), vacuum boundaries, 4 x 4 x 4 checkerboard of four seeded
materials, TT rank cap 64, truncation tolerance 1e-8, FP64, with the mixed
run of the same input next to it.  The largest configuration (1024^3 nodes,
16 groups, S16, eight materials with upscatter, rank cap 96) is measured in
the same line with a few steps (`largest_config`): one of its steps takes
tens of seconds, too long for the K-step contract of the headline.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--gpus 1]

Prints one JSON line.  `value` is power-iteration steps per second over K
timed steps (inputs resident in HBM, after W untimed steps).  The roofline
object reports the dominant kernel class timed with HIP events recorded on
the solver's stream during a second pass of K steps; `cpu_baseline` is the
plain FP64 checker (transport sweeps) timed on a bounded sample of the same
workload on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline fraction
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0

# HBM bytes per launch of a kernel class from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters scaled by a plain copy (profiles/gmres_slices_checkerboard_n128_G8_S8_traffic.md),
# valid only while the kernel's sources are unchanged.
MEASURED_TRAFFIC = {
    # HBM bytes per launch of the dominant kernel from FETCH_SIZE (scaled by
    # 2.0) plus WRITE_SIZE (scaled by 1.0) over the timed steps of a profiled
    # bench run, valid while the kernel sources hash to the prefixes below
    ("krylov", "checkerboard_n128_G8_S8"): dict(
        bytes_per_launch=1.692e9,
        sources={"paper_2309_03347_amd/csrc/krylov.hip": "53d77d2d6a5a5777",
                 "paper_2309_03347_amd/csrc/gemm_tile.h": "8641b1e5a94501dd"}),
}


def _measured_traffic(kernel, workload):
    import hashlib
    rec = MEASURED_TRAFFIC.get((kernel, workload))
    if rec is None:
        return None
    for path, prefix in rec["sources"].items():
        with open(os.path.join(ROOT, path), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest()[:16] != prefix:
                return None
    return rec["bytes_per_launch"]

WORKLOADS = {
    # name: (builder, description)
    "checkerboard_n1024_G16_S16": (lambda W: W.config(4),
                                   "1024^3 nodes, 16 groups, S16 (288 dirs), 2x2x2 blocks of 8 "
                                   "materials, upscatter in the lowest 4 groups, rank cap 96, "
                                   "tol 1e-7"),
    "checkerboard_n128_G8_S8": (lambda W: W.config(2),
                                "128^3 nodes, 8 groups, S8 (80 dirs), 4x4x4 checkerboard of 4 "
                                "materials, rank cap 64, tol 1e-8"),
    "inner_box_n32_G4_S4": (lambda W: W.config(1),
                            "32^3 nodes, 4 groups, S4 (24 dirs), two-region, rank cap 32, tol 1e-8"),
    "homogeneous_n8_S2": (lambda W: W.config(0),
                          "8^3 nodes, 1 group, S2 (8 dirs), homogeneous, rank cap 8, tol 1e-10"),
    "batch256_uneven": (None, "256 independent instances: 16^3-64^3 nodes, 1-8 groups, S2-S8, "
                              "rank caps 4-48, tol 1e-6; one batched step advances all"),
}


def _parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="checkerboard_n128_G8_S8", choices=sorted(WORKLOADS))
    p.add_argument("--rmax", type=int, default=0, help="override the rank cap (0: workload's)")
    p.add_argument("--rhs-mode", type=int, default=0, help="0 projected, 1 explicit")
    p.add_argument("--cpu-seconds", type=float, default=10.0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-probe", action="store_true")
    p.add_argument("--streams", type=int, default=4, help="streams of the batched workload")
    p.add_argument("--build-workers", type=int, default=1,
                   help="host processes building the batched workload's operators")
    p.add_argument("--instances", type=int, default=256, help="instances of the batched workload")
    p.add_argument("--no-mixed", action="store_true",
                   help="skip the mixed-precision comparison run")
    p.add_argument("--mixed-precision", type=int, default=2, choices=(2, 3),
                   help="precision of the mixed run: 2 BF16, 3 block-scaled FP16 products")
    p.add_argument("--graph-steps", type=int, default=5,
                   help="replays of the captured fixed-rank step (tt_power_step_async) after "
                        "the timed steps (0: skip)")
    p.add_argument("--graph-sweeps", type=int, default=2,
                   help="alternating sweeps of the captured fixed-rank step")
    p.add_argument("--ttk-steps", type=int, default=20,
                   help="step limit of the time-to-k run (0 skips it)")
    p.add_argument("--probe-steps", type=int, default=5,
                   help="steps of the kernel-probe pass (at most --steps)")
    p.add_argument("--largest-steps", type=int, default=2,
                   help="timed steps of the largest configuration (0 skips it)")
    p.add_argument("--largest-warmup", type=int, default=1)
    p.add_argument("--copy-calibration", action="store_true",
                   help="only copy a 256 MiB float64 device buffer three times (the plain "
                        "copy that scales the HBM traffic counters) and exit")
    return p.parse_args()


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Set the OpenMP thread count of the checker's runtime (libgomp)."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
        return True
    except OSError:
        return False


def _cpu_baseline(wl, seconds: float, host_budget_gb: float = 120.0):
    """The checker's exact power iteration on the host, timed for about
    `seconds` (at least one step), all host threads and one thread."""
    import numpy as np
    from oracle import sweep
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n_unknowns = wl.G * wl.L * wl.n ** 3
    base = dict(unit="steps/s", cores=threads, kind="oracle", cpu_model=_cpu_model())
    # the dense iteration holds about four flux-sized arrays
    need_gb = 4 * 8 * n_unknowns / 1e9
    if need_gb > host_budget_gb:
        return dict(base, value=None, single_thread=None,
                    sample=f"not runnable: one dense flux vector of this workload "
                           f"({n_unknowns:.3g} unknowns) is {8 * n_unknowns / 1e12:.1f} TB")
    prob = sweep.Problem.from_workload(wl)
    psi = sweep.dense_psi0(wl)

    def run(limit):
        nonlocal psi
        k = 1.0
        steps = 0
        t0 = time.perf_counter()
        while True:
            nxt, k = prob.power_step(psi, k)
            psi = nxt / np.linalg.norm(nxt)
            steps += 1
            dt = time.perf_counter() - t0
            if dt >= limit:
                return steps, dt

    steps, dt = run(seconds)
    single = None
    if dt / steps < 1.0 and _omp_threads(1):
        s1, d1 = run(seconds / 2)
        _omp_threads(threads)
        single = dict(value=s1 / d1, sample=f"{s1} steps in {d1:.1f} s on one thread")
    return dict(base, value=steps / dt, single_thread=single,
                sample=f"{steps} exact sweep power steps of the same workload "
                       f"({prob.n_unknowns} unknowns) in {dt:.1f} s")


def _time_to_k(wl, rmax, rhs_mode, max_steps, rel=1e-5, precision=0):
    """Wall time from the first step of a fresh solver until k stays within
    `rel` of the converged k of the same iteration (the last k when
    |dk| < tol_k, else the last k of the run, flagged unconverged).  A time is
    reported only when k then stayed within `rel` for at least five steps."""
    import torch
    from paper_2309_03347_amd.solver import KeffSolver
    s = KeffSolver(wl, rmax=rmax, rhs_mode=rhs_mode, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, ks = [], []
    converged = False
    for _ in range(max_steps):
        rec = s.step()
        times.append(time.perf_counter() - t0)
        ks.append(rec.k)
        if abs(rec.dk) < wl.tol_k:
            converged = True
            break
    s.close()
    k_ref = ks[-1]
    hit = None
    for i in range(len(ks)):
        if all(abs(k - k_ref) <= rel * abs(k_ref) for k in ks[i:]):
            hit = i
            break
    tail = ks[-10:]
    out = dict(rel=rel, k_ref=k_ref, converged=converged, steps=len(ks),
               tail_rel_spread=(max(tail) - min(tail)) / abs(k_ref))
    # A k that is still drifting by more than `rel` per step has no meaningful
    # time-to-k (a single small |dk| can stop a run whose k still wanders):
    # report null with the observed spread.
    settled = hit is not None and len(ks) - hit >= 5
    if settled and (converged or out["tail_rel_spread"] <= rel):
        out.update(seconds=times[hit], step=hit + 1)
    else:
        out.update(seconds=None, step=None)
    return out


def _build_ops(w):
    """One instance's operators, with one BLAS thread (the factorizations are
    small, and the worker processes already fill the host's cores); returns
    the operators and the build's wall and CPU seconds."""
    from threadpoolctl import threadpool_limits
    from paper_2309_03347_amd import operators
    t0, c0 = time.perf_counter(), time.process_time()
    with threadpool_limits(limits=1):
        o = operators.build(w)
    return o, time.perf_counter() - t0, time.process_time() - c0


def _batch_graph_leg(solvers, args):
    """Every instance's fixed-rank step (tt_power_step_async) captured as a
    graph of its own at its current ranks, its persistent GMRES grids capped
    at 256 / streams workgroups; one batched step replays the graphs
    round-robin on the streams, so that up to `streams` instances run at
    once (no host synchronization inside a step)."""
    import torch
    from paper_2309_03347_amd import native
    graphs, bufs, failed = [], [], []
    nst = max(1, args.streams)
    streams = [torch.cuda.Stream() for _ in range(nst)]
    torch.cuda.synchronize()
    native.set_grid_cap(256 // nst)
    for i, sv in enumerate(solvers):
        buf = native.step_info_buffer()
        g = torch.cuda.CUDAGraph()
        try:
            with torch.cuda.graph(g):
                sv.native.step_async(buf, sweeps=args.graph_sweeps)
        except Exception as e:
            failed.append((i, f"{type(e).__name__}: {e}"[:160]))
            continue
        graphs.append(g)
        bufs.append(buf)
    native.set_grid_cap(0)
    torch.cuda.synchronize()
    print(f"{len(graphs)} instance graphs captured", file=sys.stderr, flush=True)
    if not graphs:
        return dict(error="no instance step could be captured", failed=failed[:4])
    def batched_step():
        for i, g in enumerate(graphs):
            with torch.cuda.stream(streams[i % nst]):
                g.replay()

    def timed(step, label):
        step()                 # one untimed round
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(args.graph_steps):
            step()
            print(f"{label} batched step {r} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    dt = timed(batched_step, "per-instance graphs")
    infos = [native.read_step_info(b) for b in bufs]
    out = dict(value=len(graphs) * args.graph_steps / dt, unit="instance-steps/s",
               ms_per_batched_step=1e3 * dt / args.graph_steps, instances=len(graphs),
               sweeps=args.graph_sweeps, not_captured=len(failed), failed=failed[:4],
               status_counts={str(st): sum(1 for x in infos if x["status"] == st)
                              for st in sorted(set(x["status"] for x in infos))},
               streams=nst, grid_cap=256 // nst,
               note="per-instance graphs of the fixed-rank step at the ranks the adaptive "
                    "steps reached, replayed round-robin on the streams")
    return out


def _graph_leg(s, args):
    """The fixed-rank power step with no host synchronization
    (tt_power_step_async) captured once as a graph at the ranks the timed
    steps reached, then replayed: steps/s of the replays and the last
    replay's step information."""
    import torch
    from paper_2309_03347_amd import native
    buf = native.step_info_buffer()
    k0 = s.history[-1].k
    try:
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            s.native.step_async(buf, sweeps=args.graph_sweeps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.graph_steps):
            g.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    except Exception as e:           # reported, not fatal for the bench line
        return dict(error=f"{type(e).__name__}: {e}")
    info = native.read_step_info(buf)
    return dict(value=args.graph_steps / dt, unit="steps/s",
                ms_per_step=1e3 * dt / args.graph_steps, replays=args.graph_steps,
                sweeps=args.graph_sweeps, ranks="fixed at the adaptive steps' last ranks",
                k=info["k"], k_rel_diff_vs_adaptive_start=abs(info["k"] - k0) / abs(k0),
                max_local_res=info["max_local_res"], status=info["status"],
                note="one-site alternating sweeps with QR splits at fixed ranks (no truncation "
                     "or enrichment), k update and normalization on the device; one graph "
                     "launch per step")


def _roofline(probe, workload):
    """Roofline of the dominant kernel class (by total device time) of a probe."""
    name, st = max(probe.items(), key=lambda kv: kv[1]["total_ms"])
    if st["launches"] == 0:
        return None
    avg_ms = st["total_ms"] / st["launches"]
    # bound by arithmetic intensity against the ridge of the class's arithmetic
    peak_tf = PEAK_BF16_TFLOPS if name == "gemm_bf16" else PEAK_FP64_TFLOPS
    ridge = peak_tf * 1e12 / (PEAK_HBM_GBS * 1e9)
    intensity = st["flops"] / max(1.0, st["bytes"])
    if intensity >= ridge:
        achieved = st["flops"] / (st["total_ms"] * 1e-3) / 1e12
        out = dict(bound="mfma" if name == "gemm_bf16" else "alu", achieved=achieved,
                   peak=peak_tf, unit="TFLOP/s", frac=achieved / peak_tf)
    else:
        achieved = st["bytes"] / (st["total_ms"] * 1e-3) / 1e9
        out = dict(bound="hbm", achieved=achieved, peak=PEAK_HBM_GBS, unit="GB/s",
                   frac=achieved / PEAK_HBM_GBS)
    out["traffic"] = _measured_traffic(name, workload)
    out.update(kernel=name, intensity_flop_per_byte=intensity, launches=st["launches"],
               avg_us=avg_ms * 1e3, flops_per_launch=st["flops"] / st["launches"],
               bytes_per_launch=st["bytes"] / st["launches"])
    return out


def _bench_batch(args):
    """Many uneven instances advanced by tt_power_step_batched."""
    import concurrent.futures as cf
    import torch
    from paper_2309_03347_amd import workload as W
    from paper_2309_03347_amd.solver import KeffSolver, step_batched
    wls = W.batch_instances(args.instances)
    t0 = time.perf_counter()
    ops, build_wall, build_cpu = [], [], []
    def note():
        if len(ops) % 16 == 0 or len(ops) == len(wls):
            print(f"operators of {len(ops)} / {len(wls)} instances built "
                  f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    if args.build_workers > 1:
        # fresh worker processes (no threads inherited from this one), one
        # BLAS / OpenMP thread each
        import multiprocessing as mp
        keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
        prev = {k: os.environ.get(k) for k in keys}
        for k in keys:
            os.environ[k] = "1"
        ctx = mp.get_context("spawn")
        try:
            with cf.ProcessPoolExecutor(max_workers=args.build_workers, mp_context=ctx) as ex:
                for o, tw, tc in ex.map(_build_ops, wls, chunksize=2):
                    ops.append(o)
                    build_wall.append(tw)
                    build_cpu.append(tc)
                    note()
        finally:
            for k, v in prev.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
    else:
        for w in wls:
            o, tw, tc = _build_ops(w)
            ops.append(o)
            build_wall.append(tw)
            build_cpu.append(tc)
            note()
    t_ops = time.perf_counter() - t0
    print(f"operators built for {len(wls)} instances in {t_ops:.1f} s (per instance: "
          f"{sum(build_wall):.1f} s wall, {sum(build_cpu):.1f} s CPU in total)",
          file=sys.stderr, flush=True)
    solvers = []
    for w, o in zip(wls, ops):
        solvers.append(KeffSolver(w, rmax=w.rmax, ops=o))
        if len(solvers) % 32 == 0:
            print(f"{len(solvers)} solvers created ({time.perf_counter() - t0:.1f} s)",
                  file=sys.stderr, flush=True)
    setup = time.perf_counter() - t0
    print(f"solvers created in {setup - t_ops:.1f} s", file=sys.stderr, flush=True)
    streams = [torch.cuda.Stream() for _ in range(args.streams)]
    for i in range(args.warmup):
        step_batched(solvers, streams)
        print(f"warmup batched step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step_batched(solvers, streams)
        print(f"timed batched step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    graph = _batch_graph_leg(solvers, args) if args.graph_steps > 0 else None
    # kernel probe over one more batched step: every solver's launches of the
    # timed classes bracketed by HIP events on its own stream
    roofline = None
    if not args.no_probe:
        for sv in solvers:
            sv.native.set_probe(True)
        step_batched(solvers, streams)
        torch.cuda.synchronize()
        tot = {}
        for sv in solvers:
            for name, st in sv.native.probe_stats().items():
                acc = tot.setdefault(name, dict(launches=0, total_ms=0.0, flops=0.0, bytes=0.0))
                for key in acc:
                    acc[key] += st[key]
            sv.native.set_probe(False)
        roofline = _roofline(tot, "batch256_uneven")
    cpu = None
    if not args.no_cpu_baseline:
        import numpy as np
        from oracle import sweep
        # a spread sample: every 8th instance from the first, then every 8th
        # from the fourth, ... until the time budget is spent
        order = [i for off in (0, 4, 2, 6, 1, 5, 3, 7) for i in range(off, len(wls), 8)]
        steps, tc = 0, time.perf_counter()
        for i in order:
            w = wls[i]
            prob = sweep.Problem.from_workload(w)
            psi = sweep.dense_psi0(w)
            nxt, k = prob.power_step(psi, 1.0)
            steps += 1
            if time.perf_counter() - tc > args.cpu_seconds:
                break
        el = time.perf_counter() - tc
        cpu = dict(value=steps / el, unit="instance-steps/s",
                   cores=int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                   cpu_model=_cpu_model(),
                   kind="oracle",
                   sample=f"one exact power step of each of {steps} of the {len(wls)} instances "
                          f"(every 8th, spread over the batch), {el:.1f} s")
    out = {
        "metric": "power-iteration steps/sec & time-to-k at 1e-5, mixed vs FP64; TT GFLOP/s % peak",
        "value": len(solvers) * args.steps / dt,
        "unit": "instance-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded)",
        "config": {"workload": "batch256_uneven", "description": WORKLOADS["batch256_uneven"][1],
                   "instances": len(solvers), "streams": args.streams,
                   "setup_seconds": setup, "operator_build_seconds": t_ops,
                   "operator_build_cpu_seconds_summed": sum(build_cpu),
                   "build_workers": args.build_workers},
        "max_rank": int(max(max(s.native.ranks()) for s in solvers)),
        "graph_step": graph,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    for s in solvers:
        s.close()
    print("solvers closed", file=sys.stderr, flush=True)
    _teardown()


def _largest(args):
    """A few FP64 steps of the 1024^3, 16-group, S16 configuration."""
    import torch
    from paper_2309_03347_amd import workload as W
    from paper_2309_03347_amd.solver import KeffSolver
    name = "checkerboard_n1024_G16_S16"
    builder, desc = WORKLOADS[name]
    wl = builder(W)
    t0 = time.perf_counter()
    s = KeffSolver(wl)
    setup = time.perf_counter() - t0
    print(f"{name}: setup {setup:.1f} s", file=sys.stderr, flush=True)
    for i in range(args.largest_warmup):
        rec = s.step()
        print(f"{name}: warmup step {i} {rec.seconds:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.largest_steps):
        rec = s.step()
        print(f"{name}: timed step {i} {rec.seconds:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h = s.history
    out = dict(workload=name, description=desc, value=args.largest_steps / dt, unit="steps/s",
               steps=args.largest_steps, warmup=args.largest_warmup,
               ms_per_step=1e3 * dt / args.largest_steps, dtype="f64",
               unknowns=float(wl.G * wl.L * wl.n ** 3), rank_cap=wl.rmax, tol=wl.tol,
               setup_seconds=setup, k=h[-1].k, dk_last=h[-1].dk,
               max_rank=int(max(s.native.ranks())), sweeps=[r.sweeps for r in h],
               local_iters=[r.local_iters for r in h],
               cpu_baseline=_cpu_baseline(wl, args.cpu_seconds) if not args.no_cpu_baseline
               else None)
    s.close()
    return out


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the batch and "
              "single-instance paths are single-device by design.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        x = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print("copied 3 x 256 MiB", flush=True)
        return
    if args.workload == "batch256_uneven":
        return _bench_batch(args)
    import numpy as np
    import torch
    from paper_2309_03347_amd import workload as W
    from paper_2309_03347_amd.solver import KeffSolver

    builder, desc = WORKLOADS[args.workload]
    wl = builder(W)
    rmax = args.rmax or wl.rmax
    s = KeffSolver(wl, rmax=rmax, rhs_mode=args.rhs_mode)
    for i in range(args.warmup):
        s.step()
        print(f"{args.workload}: warmup step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        s.step()
        print(f"{args.workload}: timed step {i} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = args.steps / dt
    hist = s.history

    roofline = None
    probe = None
    if not args.no_probe:
        s.native.set_probe(True)
        for _ in range(max(1, min(args.steps, args.probe_steps))):
            s.step()
        torch.cuda.synchronize()
        probe = s.native.probe_stats()
        s.native.set_probe(False)
        roofline = _roofline(probe, args.workload)

    ttk = ttk_small = None
    if args.ttk_steps > 0:
        ttk = _time_to_k(wl, rmax, args.rhs_mode, args.ttk_steps)
        # The 8^3 case with the rank cap lifted (tolerance-governed ranks, the
        # regime the exact iteration is matched in): k settles, so time-to-k
        # is finite; FP64 and mixed local solves.
        small = W.config(0)
        ttk_small = dict(workload="homogeneous_n8_S2, rank cap 64 (tol 1e-10 governs)",
                         fp64=_time_to_k(small, 64, args.rhs_mode, 100),
                         mixed=_time_to_k(small, 64, args.rhs_mode, 100, precision=2))
        ttk_small["mixed_k_rel_diff_vs_fp64"] = abs(ttk_small["mixed"]["k_ref"] -
                                                    ttk_small["fp64"]["k_ref"]) / ttk_small["fp64"]["k_ref"]

    mixed = None
    if not args.no_mixed:
        # the same workload in the mixed mode: local GMRES cycles on FP32 (persistent
        # kernel) or with BF16 / FP16 matrix-core products (multi-launch GMRES), each
        # cycle refining the FP64 local residual
        sm = KeffSolver(wl, rmax=rmax, rhs_mode=args.rhs_mode, ops=s.ops,
                        precision=args.mixed_precision)
        for _ in range(args.warmup):
            sm.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sm.step()
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0
        hm = sm.history
        mixed = dict(value=args.steps / dtm, unit="steps/s", ms_per_step=1e3 * dtm / args.steps,
                     speedup_vs_fp64=(args.steps / dtm) / value, k=hm[-1].k,
                     # the FP64 solver's k after the same number of steps
                     k_rel_diff_vs_fp64=abs(hm[-1].k - hist[len(hm) - 1].k) / abs(hist[len(hm) - 1].k),
                     local_iters_last=hm[-1].local_iters,
                     fp64_local_iters_last=hist[len(hm) - 1].local_iters,
                     precision=args.mixed_precision,
                     dtype=("bf16" if args.mixed_precision == 2 else "block-scaled fp16") +
                           " matrix-core products (fp32 accumulation) and fp32 Krylov "
                           "cycles in refined local solves; fp64 residuals, interfaces, "
                           "QR / SVD, k")
        sm.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(wl, args.cpu_seconds)

    graph = None
    if args.graph_steps > 0:
        graph = _graph_leg(s, args)
    largest = None
    if args.largest_steps > 0 and args.workload != "checkerboard_n1024_G16_S16":
        largest = _largest(args)

    out = {
        "metric": "power-iteration steps/sec & time-to-k at 1e-5, mixed vs FP64; TT GFLOP/s % peak",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": args.workload, "description": desc, "rank_cap": rmax,
                   "tol": wl.tol, "rhs_mode": "projected" if args.rhs_mode == 0 else "explicit",
                   "unknowns": int(wl.G * wl.L * wl.n ** 3),
                   "quadrature": "level-symmetric points, LQn weights"},
        "k": hist[-1].k,
        "dk_last": hist[-1].dk,
        "max_rank": int(max(s.native.ranks())),
        "sweeps_last": hist[-1].sweeps,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "time_to_k": ttk,
        "time_to_k_small": ttk_small,
        "mixed": mixed,
        "graph_step": graph,
        "largest_config": largest,
    }
    if probe is not None:
        out["kernel_probe"] = {k: dict(launches=v["launches"], ms=round(v["total_ms"], 3))
                               for k, v in probe.items() if v["launches"]}
    print(json.dumps(out), flush=True)
    s.close()
    _teardown()


def _teardown():
    """Orderly end: wait for the device and free the library's per-thread
    resources before the interpreter and the HIP runtime shut down."""
    import torch
    from paper_2309_03347_amd import native
    torch.cuda.synchronize()
    native.release()


if __name__ == "__main__":
    main()
