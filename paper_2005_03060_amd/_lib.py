"""ctypes declarations for librrcal.so (include/rrcal.h).

The shared library is built in-tree by `paper_2005_03060_amd.build`; there
is no fallback: a missing library raises at load time.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librrcal.so")

RRC_OK = 0
RRC_EINVAL = -1
RRC_EDEGEN = -2
RRC_EDEVICE = -3
RRC_ENOTIMPL = -4
RRC_ERANGE = -5

RRC_C64 = 0
RRC_CI4 = 1
RRC_INIT_FIRSTCAL = 0
RRC_INIT_GAINS = 1
RRC_DEGEN_REFANT = 0
RRC_DEGEN_MATCH = 1
RRC_RUN_PIPELINED = 1
RRC_RUN_SELFCAL = 2
RRC_ORDER_XENG_FIRST = 0
RRC_ORDER_FFT_FIRST = 1
RRC_ORDER_SERIAL = 2
RRC_BATCH_GRAPH = 1
RRC_XENG_AUTO = 0
RRC_XENG_DOT = 1
RRC_XENG_MFMA = 2
RRC_MAX_TYPES = 16
RRC_MAX_GRID = 64
RRC_STATIC_SCRATCH_BYTES = 32 << 20
RRC_LOWCAD_MAX_GRID = 32
RRC_LOWCAD_MAX_CYCLES = 256
RRC_METRIC_SQUARE = 0
RRC_METRIC_HEX = 1

EXPORTS = ("rrc_default_opts", "rrc_select_subset", "rrc_degeneracy_count", "rrc_plan_create",
           "rrc_plan_destroy", "rrc_plan_get_info", "rrc_workspace_size", "rrc_fftcorr",
           "rrc_xengine", "rrc_solve", "rrc_chisq_fwd", "rrc_chisq_adj", "rrc_run", "rrc_strerror",
           "rrc_batch_create", "rrc_batch_destroy", "rrc_batch_run", "rrc_plan_prepare",
           "rrc_plan_set_order", "rrc_wall_clock_hz", "rrc_run_static", "rrc_plan_set_xengine",
           "rrc_gain_variance", "rrc_omnical", "rrc_lowcad_schedule", "rrc_lowcad_xengine",
           "rrc_lowcad_solve", "rrc_plan_tune", "rrc_hex_mask", "rrc_select_subset_masked",
           "rrc_degeneracy_count_masked", "rrc_plan_create_masked", "rrc_chisq_full",
           "rrc_plan_set_fft_size")


class SolverOpts(C.Structure):
    _fields_ = [("init_mode", C.c_int32), ("degen_mode", C.c_int32), ("max_gn", C.c_int32),
                ("fp64_steps", C.c_int32), ("max_cg", C.c_int32), ("cg_tol", C.c_float),
                ("tol32", C.c_float)]


class PlanInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_ant", C.c_int32), ("fft_size", C.c_int32),
                ("n_lags", C.c_int32), ("n_types", C.c_int32), ("n_pairs", C.c_int32),
                ("dof", C.c_int32), ("n_units", C.c_int32), ("n_time", C.c_int32),
                ("dtype", C.c_int32), ("workspace_bytes", C.c_uint64), ("n_live", C.c_int32),
                ("masked", C.c_int32)]


class RunIO(C.Structure):
    _fields_ = [("d_volt", C.c_void_p), ("d_gains_in", C.c_void_p), ("d_gains_ref", C.c_void_p),
                ("d_vunique", C.c_void_p), ("d_vauto", C.c_void_p), ("d_vred", C.c_void_p),
                ("d_gains_out", C.c_void_p), ("d_vmodel", C.c_void_p), ("d_chisq", C.c_void_p),
                ("d_niter", C.c_void_p), ("d_status", C.c_void_p), ("d_work", C.c_void_p),
                ("d_stamps", C.c_void_p)]


class Tune(C.Structure):
    _fields_ = [("fft_chunk_factor", C.c_int32), ("order", C.c_int32), ("xengine", C.c_int32),
                ("ms_per_run", C.c_float), ("from_cache", C.c_int32), ("fft_size", C.c_int32)]


class RRCError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


_LIB = None


def load_library() -> C.CDLL:
    """Loads librrcal.so once; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2005_03060_amd.build` "
                           "(there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, pi32, pf = C.c_void_p, C.c_int32, C.POINTER(C.c_int32), C.c_void_p
    sig = {
        "rrc_default_opts": (None, [C.POINTER(SolverOpts)]),
        "rrc_select_subset": (C.c_int, [i32, C.c_double, C.c_double, pi32, i32, pi32, pi32]),
        "rrc_degeneracy_count": (C.c_int, [i32, pi32, i32, pi32, pi32]),
        "rrc_plan_create": (C.c_int, [C.POINTER(vp), i32, pi32, i32, i32, i32, i32,
                                      C.POINTER(SolverOpts)]),
        "rrc_plan_destroy": (None, [vp]),
        "rrc_plan_get_info": (C.c_int, [vp, C.POINTER(PlanInfo)]),
        "rrc_workspace_size": (C.c_int, [vp, C.POINTER(C.c_size_t)]),
        "rrc_fftcorr": (C.c_int, [vp, vp, vp, vp, vp, pf, vp]),
        "rrc_xengine": (C.c_int, [vp, vp, vp, vp, vp]),
        "rrc_solve": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, pf, vp, vp, vp]),
        "rrc_chisq_fwd": (C.c_int, [vp, vp, vp, vp, vp, pf]),
        "rrc_chisq_adj": (C.c_int, [vp, vp, vp, vp, vp, vp, vp, pf, pf]),
        "rrc_run": (C.c_int, [vp, vp, i32, C.POINTER(RunIO)]),
        "rrc_strerror": (C.c_char_p, [C.c_int]),
        "rrc_batch_create": (C.c_int, [C.POINTER(vp), i32, C.POINTER(vp), C.c_uint32]),
        "rrc_batch_destroy": (None, [vp]),
        "rrc_batch_run": (C.c_int, [vp, vp, i32, C.POINTER(RunIO)]),
        "rrc_plan_prepare": (C.c_int, [vp]),
        "rrc_plan_set_order": (C.c_int, [vp, i32]),
        "rrc_wall_clock_hz": (C.c_int, [C.POINTER(C.c_double)]),
        "rrc_run_static": (C.c_int, [vp, vp, i32, C.POINTER(RunIO)]),
        "rrc_plan_set_xengine": (C.c_int, [vp, i32]),
        "rrc_gain_variance": (C.c_int, [i32, pi32, i32, C.c_double, C.POINTER(C.c_double)]),
        "rrc_omnical": (C.c_int, [vp, vp, vp, vp, i32, C.c_float, i32, vp, vp, pf, vp, vp, pf, vp]),
        "rrc_hex_mask": (C.c_int, [i32, vp, i32, pi32, pi32]),
        "rrc_chisq_full": (C.c_int, [i32, i32, vp, vp, vp, vp, vp, vp]),
        "rrc_plan_set_fft_size": (C.c_int, [vp, i32]),
        "rrc_select_subset_masked": (C.c_int, [i32, vp, i32, C.c_double, C.c_double, pi32, i32, pi32, pi32]),
        "rrc_degeneracy_count_masked": (C.c_int, [i32, vp, pi32, i32, pi32, pi32]),
        "rrc_plan_create_masked": (C.c_int, [C.POINTER(vp), i32, vp, pi32, i32, i32, i32, i32,
                                             C.POINTER(SolverOpts)]),
        "rrc_lowcad_schedule": (C.c_int, [i32, C.c_double, C.c_double, pi32, i32, pi32]),
        "rrc_plan_tune": (C.c_int, [vp, vp, C.POINTER(RunIO), C.c_char_p, C.POINTER(Tune)]),
        "rrc_lowcad_xengine": (C.c_int, [i32, i32, i32, pi32, i32, vp, vp, vp]),
        "rrc_lowcad_solve": (C.c_int, [i32, i32, vp, vp, vp, i32, C.c_float, vp, vp, pf, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def strerror(code: int) -> str:
    if _LIB is None:
        return f"error {code}"
    return _LIB.rrc_strerror(code).decode()


def check(code: int, where: str) -> None:
    if code != RRC_OK:
        raise RRCError(code, where)
