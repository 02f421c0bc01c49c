"""C-ABI contract checks that need no GPU: symbols and host-side validation."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2309_03347_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ttnt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(tt[a-z_]*|ttnt_version)\s*\(", text)
    return sorted(set(n for n in names if n not in ("tt_status",)))


def test_library_exports_every_declared_symbol():
    lib = native.lib()
    declared = _declared()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(native.EXPORTED)
    assert lib.ttnt_version() == 10000


def _host_vec(n, r, rcap):
    n = np.array(n, dtype=np.int32)
    r = np.array(r, dtype=np.int32)
    rcap = np.array(rcap, dtype=np.int32)
    off = np.zeros(len(n), dtype=np.int64)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    v = native.TTVec(len(n), n.ctypes.data_as(native.I32P), r.ctypes.data_as(native.I32P),
                     rcap.ctypes.data_as(native.I32P), fake, off.ctypes.data_as(native.I64P))
    return v, (n, r, rcap, off)


def _host_mat(m, n, R):
    m = np.array(m, dtype=np.int32)
    n = np.array(n, dtype=np.int32)
    R = np.array(R, dtype=np.int32)
    off = np.zeros(len(m), dtype=np.int64)
    A = native.TTMat(len(m), m.ctypes.data_as(native.I32P), n.ctypes.data_as(native.I32P),
                     R.ctypes.data_as(native.I32P), ctypes.c_void_p(0x1000),
                     off.ctypes.data_as(native.I64P))
    return A, (m, n, R, off)


def test_matvec_rejects_mismatched_modes():
    lib = native.lib()
    A, ka = _host_mat([2, 2], [2, 3], [1, 2, 1])
    x, kx = _host_vec([2, 2], [1, 2, 1], [1, 2, 1])
    y, ky = _host_vec([2, 2], [1, 1, 1], [1, 4, 1])
    st = lib.tt_matvec(ctypes.byref(A), ctypes.byref(x), ctypes.byref(y), None)
    assert st == native.TT_E_ARG
    assert b"modes" in lib.tt_last_error()


def test_matvec_reports_capacity():
    lib = native.lib()
    A, ka = _host_mat([2, 2], [2, 2], [1, 3, 1])
    x, kx = _host_vec([2, 2], [1, 2, 1], [1, 2, 1])
    y, ky = _host_vec([2, 2], [1, 1, 1], [1, 5, 1])   # needs 6
    assert lib.tt_matvec(ctypes.byref(A), ctypes.byref(x), ctypes.byref(y), None) == native.TT_E_CAPACITY
    assert ky[1].tolist() == [1, 1, 1]    # nothing written


def test_round_rejects_bad_arguments():
    lib = native.lib()
    x, kx = _host_vec([2, 2], [1, 3, 1], [1, 2, 1])    # rank above capacity
    st = lib.tt_round(ctypes.byref(x), 1e-8, 4, None, ctypes.c_void_p(0x1000), 1 << 20, None)
    assert st == native.TT_E_ARG
    x, kx = _host_vec([2, 2], [1, 2, 1], [1, 2, 1])
    st = lib.tt_round(ctypes.byref(x), -1.0, 4, None, ctypes.c_void_p(0x1000), 1 << 20, None)
    assert st == native.TT_E_ARG
    st = lib.tt_round(ctypes.byref(x), 1e-8, 0, None, ctypes.c_void_p(0x1000), 1 << 20, None)
    assert st == native.TT_E_ARG
    st = lib.tt_round(ctypes.byref(x), 1e-8, 4, None, ctypes.c_void_p(0x1000), 8, None)
    assert st == native.TT_E_CAPACITY


def test_local_solve_rejects_non_square():
    lib = native.lib()
    sysd = native.TTLocal(2, 1, 2, 3, 1, 2, ctypes.c_void_p(8), ctypes.c_void_p(8),
                          ctypes.c_void_p(8), ctypes.c_void_p(8))
    opts = native.TTSolveOpts(0, 1e-10, 10, 10, 64)
    info = native.TTSolveInfo()
    st = lib.tt_local_solve(ctypes.byref(sysd), ctypes.c_void_p(8), ctypes.byref(opts),
                            ctypes.byref(info), ctypes.c_void_p(8), 1 << 30, None)
    assert st == native.TT_E_ARG


def test_local_solve_rejects_unknown_method():
    lib = native.lib()
    sysd = native.TTLocal(2, 1, 3, 3, 1, 2, ctypes.c_void_p(8), ctypes.c_void_p(8),
                          ctypes.c_void_p(8), ctypes.c_void_p(8))
    info = native.TTSolveInfo()
    for method in (-1, 5):
        opts = native.TTSolveOpts(method, 1e-10, 10, 10, 64)
        st = lib.tt_local_solve(ctypes.byref(sysd), ctypes.c_void_p(8), ctypes.byref(opts),
                                ctypes.byref(info), ctypes.c_void_p(8), 1 << 30, None)
        assert st == native.TT_E_ARG, method
        assert b"method" in native.lib().tt_last_error()


def test_precision_outside_the_defined_modes_is_rejected():
    # 0 FP64, 1 mixed, 2 BF16 products, 3 block-scaled FP16 products; the
    # product alone has no mode 1
    lib = native.lib()
    sysd = native.TTLocal(2, 1, 3, 3, 1, 2, ctypes.c_void_p(8), ctypes.c_void_p(8),
                          ctypes.c_void_p(8), ctypes.c_void_p(8))
    info = native.TTSolveInfo()
    for precision in (-1, 4):
        opts = native.TTSolveOpts(0, 1e-10, 10, 10, 64, precision)
        st = lib.tt_local_solve(ctypes.byref(sysd), ctypes.c_void_p(8), ctypes.byref(opts),
                                ctypes.byref(info), ctypes.c_void_p(8), 1 << 30, None)
        assert st == native.TT_E_ARG, precision
        assert b"precision" in lib.tt_last_error()
    for precision in (-1, 1, 4):
        st = lib.tt_local_apply(ctypes.byref(sysd), ctypes.c_void_p(8), ctypes.c_void_p(8),
                                precision, ctypes.c_void_p(8), 1 << 30, None)
        assert st == native.TT_E_ARG, precision
        assert b"precision" in lib.tt_last_error()
    H, kh = _host_mat([2], [2], [1, 1])
    SF, ks = _host_mat([2], [2], [1, 1])
    cF, kc = _host_vec([2], [1, 1], [1, 1])
    p0, kp = _host_vec([2], [1, 1], [1, 1])
    prob = native.TTProblem(H, SF, ctypes.c_void_p(0x1000), cF, p0, 1.0)
    opts = native.TTSolverOpts(1e-8, 4, 4, 10, 0, 0, 0.0, 40, 100, 64, 4)
    h = ctypes.c_void_p()
    assert lib.tt_solver_create(ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(h)) == native.TT_E_ARG
    assert b"precision" in lib.tt_last_error()


def test_solver_rejects_bad_options():
    lib = native.lib()
    H, kh = _host_mat([2], [2], [1, 1])
    SF, ks = _host_mat([2], [2], [1, 1])
    cF, kc = _host_vec([2], [1, 1], [1, 1])
    p0, kp = _host_vec([2], [1, 1], [1, 1])
    prob = native.TTProblem(H, SF, ctypes.c_void_p(0x1000), cF, p0, 1.0)
    opts = native.TTSolverOpts(1e-8, 0, 4, 10, 0, 0, 0.0, 40, 100, 64)   # rmax = 0
    h = ctypes.c_void_p()
    assert lib.tt_solver_create(ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(h)) == native.TT_E_ARG
    opts = native.TTSolverOpts(1e-8, 4, 4, 10, 7, 0, 0.0, 40, 100, 64)   # bad rhs_mode
    assert lib.tt_solver_create(ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(h)) == native.TT_E_ARG
    for field, bad in [("cap_eta", 1.5), ("stall", 2.0), ("min_sweeps", -1)]:
        opts = native.TTSolverOpts(1e-8, 4, 4, 10, 0, 0, 0.0, 40, 100, 64)
        setattr(opts, field, bad)
        assert lib.tt_solver_create(ctypes.byref(prob), ctypes.byref(opts),
                                    ctypes.byref(h)) == native.TT_E_ARG, field
        assert b"sweep-stopping" in lib.tt_last_error()
    prob = native.TTProblem(H, SF, ctypes.c_void_p(0x1000), cF, p0, -1.0)  # k0 <= 0
    opts = native.TTSolverOpts(1e-8, 4, 4, 10, 0, 0, 0.0, 40, 100, 64)
    assert lib.tt_solver_create(ctypes.byref(prob), ctypes.byref(opts), ctypes.byref(h)) == native.TT_E_ARG


def test_solver_workspace_query_validates_before_reading_the_device():
    lib = native.lib()
    H, kh = _host_mat([2], [2], [1, 1])
    SF, ks = _host_mat([2], [2], [1, 1])
    cF, kc = _host_vec([2], [1, 1], [1, 1])
    p0, kp = _host_vec([2], [1, 1], [1, 1])
    prob = native.TTProblem(H, SF, ctypes.c_void_p(0x1000), cF, p0, 1.0)
    good = native.TTSolverOpts(1e-8, 4, 4, 10, 0, 0, 0.0, 40, 100, 64)
    bad = native.TTSolverOpts(1e-8, 0, 4, 10, 0, 0, 0.0, 40, 100, 64)    # rmax = 0
    nbytes = ctypes.c_size_t(0)
    assert lib.tt_solver_workspace_size(None, ctypes.byref(good),
                                        ctypes.byref(nbytes)) == native.TT_E_ARG
    assert lib.tt_solver_workspace_size(ctypes.byref(prob), ctypes.byref(good),
                                        None) == native.TT_E_ARG
    assert lib.tt_solver_workspace_size(ctypes.byref(prob), ctypes.byref(bad),
                                        ctypes.byref(nbytes)) == native.TT_E_ARG
    h = ctypes.c_void_p()
    assert lib.tt_solver_create_in(ctypes.byref(prob), ctypes.byref(good), None, 0,
                                   ctypes.byref(h)) == native.TT_E_ARG
    assert b"workspace" in lib.tt_last_error()
    assert lib.tt_solver_create_in(ctypes.byref(prob), ctypes.byref(bad), ctypes.c_void_p(0x1000),
                                   1 << 20, ctypes.byref(h)) == native.TT_E_ARG


def test_async_step_validates_arguments():
    lib = native.lib()
    assert lib.tt_power_step_async(None, 0, ctypes.c_void_p(0x1000), None) == native.TT_E_ARG
    assert lib.tt_power_step_async(ctypes.c_void_p(0x1000), 0, None, None) == native.TT_E_ARG
    assert b"NULL" in lib.tt_last_error()
    assert lib.tt_power_step_async(ctypes.c_void_p(0x1000), -1, ctypes.c_void_p(0x1000),
                                   None) == native.TT_E_ARG


def test_batched_step_validates_arguments():
    lib = native.lib()
    infos = (native.TTStepInfo * 2)()
    streams = (ctypes.c_void_p * 1)(None)
    assert lib.tt_power_step_batched(None, 0, None, None, 0) == native.TT_OK   # empty batch
    assert lib.tt_power_step_batched(None, -1, infos, streams, 1) == native.TT_E_ARG
    nulls = (ctypes.c_void_p * 2)(None, None)
    assert lib.tt_power_step_batched(nulls, 2, infos, streams, 0) == native.TT_E_ARG
    assert lib.tt_power_step_batched(nulls, 2, infos, streams, 1) == native.TT_E_ARG
    assert b"NULL solver" in lib.tt_last_error()
    twice = (ctypes.c_void_p * 2)(0x1000, 0x1000)     # never dereferenced: rejected first
    assert lib.tt_power_step_batched(twice, 2, infos, streams, 1) == native.TT_E_ARG
    assert b"twice" in lib.tt_last_error()


def test_noalloc_local_solve_rejects_systems_above_its_scratch():
    # 64 MiB of static scratch: a 2 x 300 x 300 dense system needs far more
    # workspace, so the call fails before touching the device.
    lib = native.lib()
    fake = ctypes.c_void_p(0x1000)
    sysd = native.TTLocal(300, 4, 2, 2, 4, 300, fake, fake, fake, fake)
    opts = native.TTSolveOpts(1, 1e-12, 100, 40, 1 << 30, 0)
    info = native.TTSolveInfo()
    st = lib.tt_local_solve_noalloc(ctypes.byref(sysd), fake, ctypes.byref(opts),
                                    ctypes.byref(info), None)
    assert st == native.TT_E_CAPACITY
    assert b"static scratch" in lib.tt_last_error()


def test_local_apply_validates_before_launch():
    lib = native.lib()
    fake = ctypes.c_void_p(0x1000)
    sysd = native.TTLocal(3, 2, 2, 2, 2, 3, fake, fake, fake, None)
    ws = lib.tt_local_apply_workspace(ctypes.byref(sysd))
    assert ws > 0
    assert lib.tt_local_apply(ctypes.byref(sysd), fake, fake, 1, fake, ws, None) == native.TT_E_ARG
    assert lib.tt_local_apply(ctypes.byref(sysd), fake, fake, 0, fake, 8, None) == native.TT_E_CAPACITY
