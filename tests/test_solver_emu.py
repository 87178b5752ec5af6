"""The solver kernel's workgroup body, compiled for the CPU (each work-item
a fiber, barriers and wave shuffles emulated), against the FP64 oracle.

This exercises the HIP source itself without a GPU: indexing, barriers
(a non-uniform barrier is reported), the Gauss-Newton/CG logic and the
FP64 refinement and degeneracy fixing."""
import ctypes as C
import hashlib
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import correlator as OC
from oracle import geometry as OG
from oracle import redcal as OR
from tests.gpu_util import TOL_GAINS, make_units

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu", "solve_emu.cpp")
DEPS = [SRC] + [os.path.join(HERE, "..", "paper_2005_03060_amd", "csrc", f)
                for f in ("solve.hip", "rrc_device.h", "rrc_launch.h", "rrc_emu.h")]


@pytest.fixture(scope="session")
def emu():
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    h = hashlib.sha1(b"".join(open(p, "rb").read() for p in DEPS)).hexdigest()[:16]
    out = os.path.join(tempfile.gettempdir(), f"rrc_solve_emu_{h}.so")
    if not os.path.exists(out):
        tmp = out + f".{os.getpid()}.tmp"
        subprocess.run([cxx, "-std=c++17", "-O1", "-shared", "-fPIC", "-w", "-x", "c++", SRC, "-o", tmp],
                       check=True)
        os.replace(tmp, out)
    return C.CDLL(out)


def emu_solve(lib, vred, n, types, init=0, degen=0, gin=None, gref=None, threads=0, max_gn=12, fp64=1,
              max_cg=400, cg_tol=1e-2, tol32=1e-5, order=0, vcache=1):
    U = vred.shape[0]
    N, K = n * n, len(types)
    txy = (C.c_int * (2 * K))(*[v for t in types for v in t])
    io = (C.c_int * 5)(init, degen, max_gn, fp64, max_cg)
    fo = (C.c_float * 2)(cg_tol, tol32)
    vr = np.ascontiguousarray(vred.astype(np.complex64))
    go = np.zeros((U, N), np.complex64)
    vm = np.zeros((U, K), np.complex64)
    ch = np.zeros(U, np.float32)
    ni = np.zeros(U, np.int32)
    st = np.zeros(U, np.int32)

    def p(a):
        return None if a is None else a.ctypes.data_as(C.c_void_p)

    rc = lib.rrc_emu_solve(n, txy, K, U, 0, p(vr), p(gin), p(gref), io, fo, p(go), p(vm),
                           ch.ctypes.data_as(C.POINTER(C.c_float)), ni.ctypes.data_as(C.POINTER(C.c_int)),
                           st.ctypes.data_as(C.POINTER(C.c_int)), threads, order, vcache)
    assert rc == 0, "non-uniform barrier" if rc == -2 else rc
    return go, vm, ch, ni, st


def _vred(n, T, seed_wid=90, snr=10.0):
    v, g = make_units(n, 1, T, wid=seed_wid, snr=snr)
    pos = OG.square_positions(n)
    types = OG.select_subset_square(n)
    pairs, tix = OG.group_pairs(pos, types)
    vr = OC.xengine(OC.fx_correlate(v[0].astype(np.complex128)), pairs).astype(np.complex64)[None]
    return vr, g, pos, types, pairs, tix


# workgroup shapes: 256 (one wave per SIMD, direct reduction), 64 with four
# antennas per work-item, 1024 (two-level reduction, most work-items idle)
@pytest.mark.parametrize("n,threads,vcache", [(8, 0, 1), (12, 64, 1), (8, 1024, 1), (8, 0, 0), (12, 64, 0)])
def test_emulated_solver_matches_oracle(emu, n, threads, vcache):
    vr, _, pos, types, pairs, tix = _vred(n, 256)
    go, vm, ch, ni, st = emu_solve(emu, vr, n, types, threads=threads, vcache=vcache)
    ref = OR.calibrate(vr[0].astype(np.complex128), pos, types, pairs, tix)
    assert st[0] == 0
    assert np.max(np.abs(go[0] - ref["g"]) / np.abs(ref["g"])) <= TOL_GAINS
    assert np.max(np.abs(vm[0] - ref["vm"]) / np.abs(ref["vm"])) <= 1e-5
    assert abs(ch[0] - ref["chisq"]) <= 1e-5 * ref["chisq"]


def test_emulated_solver_ragged_grid_and_match(emu):
    n = 7
    vr, g, pos, types, pairs, tix = _vred(n, 150, snr=20.0)
    gin = g.astype(np.complex64)
    go, _, _, _, st = emu_solve(emu, vr, n, types, init=1, degen=1, gin=gin, gref=gin)
    g0 = gin[0].astype(np.complex128)
    ref = OR.calibrate(vr[0].astype(np.complex128), pos, types, pairs, tix, fix="match", g_ref=g0,
                       init=(g0, OR.group_mean(vr[0].astype(np.complex128), g0, pairs, tix, len(types))))
    assert st[0] == 0
    assert np.max(np.abs(go[0] - ref["g"]) / np.abs(ref["g"])) <= TOL_GAINS


def test_emulated_solver_flags_nonfinite(emu):
    vr, _, pos, types, pairs, tix = _vred(6, 64)
    vr[0, 3] = np.nan
    _, _, _, _, st = emu_solve(emu, vr, 6, types)
    assert st[0] == 2


def test_emulated_solver_maxiter_status(emu):
    vr, _, pos, types, pairs, tix = _vred(6, 64)
    _, _, _, ni, st = emu_solve(emu, vr, 6, types, max_gn=1, fp64=0)
    assert st[0] == 1 and ni[0] == 1


@pytest.mark.parametrize("n,threads", [(8, 0), (10, 64)])
def test_emulated_solver_has_no_data_race(emu, n, threads):
    # the result must not depend on the order work-items run between barriers
    vr, _, pos, types, pairs, tix = _vred(n, 256)
    outs = [emu_solve(emu, vr, n, types, threads=threads, order=o) for o in (0, 1, 2)]
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
