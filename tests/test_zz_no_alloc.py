"""rrc_run_static (no workspace: the library's static device scratch)
against rrc_run with a caller workspace, through the C-ABI: two calls in a
row on one GPU, the second with a smaller input, each bit for bit equal to
the workspace path (same kernels, deterministic reductions)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2005_03060_amd import _lib as L
from tests.gpu_util import make_ci4_units, make_units

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda")
KEYS = ("vunique", "vauto", "vred", "gains", "vmodel", "chisq", "niter", "status")


def _case(rrc, n, U, T, dtype):
    if dtype == "ci4":
        b, _, _, g = make_ci4_units(n, U, T, wid=400 + n)
        v = torch.from_numpy(b).to(DEV)
    else:
        vv, g = make_units(n, U, T, wid=400 + n)
        v = torch.from_numpy(vv).to(DEV)
    types, _ = rrc.select_subset(n)
    plan = rrc.Plan(n, types, U, T, dtype=dtype)
    return plan, v, torch.from_numpy(g.astype(np.complex64)).to(DEV)


def _static_call(lib, plan, v, gin, mode):
    out = plan.alloc_outputs(DEV)
    io = plan.run_io(v, gin, None, out)
    io.d_work = None
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = {"pipelined": L.RRC_RUN_PIPELINED, "selfcal": L.RRC_RUN_SELFCAL}[mode]
    rc = lib.rrc_run_static(plan._h, stream, code, C.byref(io))
    assert rc == L.RRC_OK, lib.rrc_strerror(rc)
    return out


@pytest.mark.parametrize("mode", ["pipelined", "selfcal"])
def test_static_run_matches_workspace_run(rrc, mode):
    lib = L.load_library()
    # larger first (16x16, 64 channels, 1024 samples: the 20 MB workspace
    # of the benchmark's complex64 workload), then a smaller 4-bit one
    cases = [(16, 64, 1024, "c64"), (12, 3, 300, "ci4")]
    for n, U, T, dtype in cases:
        plan, v, gin = _case(rrc, n, U, T, dtype)
        assert plan.info["workspace_bytes"] <= L.RRC_STATIC_SCRATCH_BYTES
        ref = plan.run(v, gains_in=gin, mode=mode)
        torch.cuda.synchronize()
        plan.prepare()
        got = _static_call(lib, plan, v, gin, mode)
        torch.cuda.synchronize()
        for k in KEYS:
            assert torch.equal(got[k], ref[k]), (n, dtype, mode, k)


def test_static_run_refusals(rrc):
    lib = L.load_library()
    # a plan whose workspace exceeds the scratch
    n, U, T = 32, 16, 2048
    types, _ = rrc.select_subset(n)
    big = rrc.Plan(n, types, U, T)
    assert big.info["workspace_bytes"] > L.RRC_STATIC_SCRATCH_BYTES
    big.prepare()
    vol = torch.empty((U, T, n * n), dtype=torch.complex64, device=DEV)
    gin = torch.ones((U, n * n), dtype=torch.complex64, device=DEV)
    out = big.alloc_outputs(DEV)
    io = big.run_io(vol, gin, None, out)
    io.d_work = None
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.rrc_run_static(big._h, stream, L.RRC_RUN_PIPELINED, C.byref(io)) == L.RRC_ERANGE
    # a workspace passed in, and a plan not yet prepared
    plan, v, g = _case(rrc, 8, 1, 64, "c64")
    out = plan.alloc_outputs(DEV)
    io = plan.run_io(v, g, None, out)
    assert lib.rrc_run_static(plan._h, stream, L.RRC_RUN_PIPELINED, C.byref(io)) == L.RRC_EINVAL
    io.d_work = None
    assert lib.rrc_run_static(plan._h, stream, L.RRC_RUN_PIPELINED, C.byref(io)) == L.RRC_EINVAL
