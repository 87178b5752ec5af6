"""Python surface over the C-ABI: argument marshalling only.

Every step of the path runs in the HIP kernels of librrcal.so; PyTorch
provides device memory (all buffers, including the workspace) and the
current stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import _lib as L


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _types_array(types: Sequence[Tuple[int, int]]):
    flat = [int(v) for d in types for v in d]
    return (C.c_int32 * max(1, len(flat)))(*flat)


def select_subset(n: int, p: float = 1.0, log_base: float = 0.0):
    """Subset selection rule (host only): returns (types, n_pairs)."""
    lib = L.load_library()
    buf = (C.c_int32 * (2 * L.RRC_MAX_TYPES))()
    k, npairs = C.c_int32(), C.c_int32()
    L.check(lib.rrc_select_subset(n, p, log_base, buf, L.RRC_MAX_TYPES, C.byref(k), C.byref(npairs)),
            "rrc_select_subset")
    return [(buf[2 * t], buf[2 * t + 1]) for t in range(k.value)], npairs.value


def degeneracy_count(n: int, types: Sequence[Tuple[int, int]]):
    """(amplitude, phase) null-space dimensions of a selection (host only)."""
    lib = L.load_library()
    na, nph = C.c_int32(), C.c_int32()
    L.check(lib.rrc_degeneracy_count(n, _types_array(types), len(types), C.byref(na), C.byref(nph)),
            "rrc_degeneracy_count")
    return na.value, nph.value


def hex_mask(side: int):
    """The hexagon of `side` antennas per edge on its (2 side - 1)^2 lattice
    grid (host only): returns (n, mask uint8 [n*n] numpy array)."""
    import numpy as np
    lib = L.load_library()
    n_max = 2 * side - 1
    mask = np.zeros(max(1, n_max * n_max), dtype=np.uint8)
    n, live = C.c_int32(), C.c_int32()
    L.check(lib.rrc_hex_mask(int(side), mask.ctypes.data, mask.size, C.byref(n), C.byref(live)), "rrc_hex_mask")
    return n.value, mask[: n.value * n.value]


def _mask_arg(n: int, mask):
    import numpy as np
    m = np.ascontiguousarray(np.asarray(mask, dtype=np.uint8).reshape(-1))
    if m.size != n * n:
        raise ValueError(f"mask must hold n*n = {n * n} entries")
    return m


def select_subset_masked(n: int, mask, metric: str = "hex", p: float = 1.0, log_base: float = 0.0):
    """Subset selection on a masked lattice (host only): (types, n_pairs)."""
    lib = L.load_library()
    m = _mask_arg(n, mask)
    buf = (C.c_int32 * (2 * L.RRC_MAX_TYPES))()
    k, npairs = C.c_int32(), C.c_int32()
    met = {"square": L.RRC_METRIC_SQUARE, "hex": L.RRC_METRIC_HEX}[metric]
    L.check(lib.rrc_select_subset_masked(n, m.ctypes.data, met, p, log_base, buf, L.RRC_MAX_TYPES, C.byref(k),
                                         C.byref(npairs)), "rrc_select_subset_masked")
    return [(buf[2 * t], buf[2 * t + 1]) for t in range(k.value)], npairs.value


def degeneracy_count_masked(n: int, mask, types: Sequence[Tuple[int, int]]):
    """(amplitude, phase) null-space dimensions on a masked lattice (host only)."""
    lib = L.load_library()
    m = _mask_arg(n, mask)
    na, nph = C.c_int32(), C.c_int32()
    L.check(lib.rrc_degeneracy_count_masked(n, m.ctypes.data, _types_array(types), len(types), C.byref(na),
                                            C.byref(nph)), "rrc_degeneracy_count_masked")
    return na.value, nph.value


def gain_variance(n: int, types: Sequence[Tuple[int, int]], snr: float):
    """Predicted per-antenna E|g_est/g_true - 1|^2 of a selection (host only)."""
    import numpy as np
    lib = L.load_library()
    out = np.empty(n * n, dtype=np.float64)
    L.check(lib.rrc_gain_variance(n, _types_array(types), len(types), float(snr),
                                  out.ctypes.data_as(C.POINTER(C.c_double))), "rrc_gain_variance")
    return out


def lowcad_schedule(n: int, p: float = 1.0, log_base: float = 0.0):
    """Low-cadence round robin (host only): list of cycles as lag-order type
    ranges (t0, t1)."""
    lib = L.load_library()
    buf = (C.c_int32 * (L.RRC_LOWCAD_MAX_CYCLES + 1))()
    nc = C.c_int32()
    L.check(lib.rrc_lowcad_schedule(n, p, log_base, buf, L.RRC_LOWCAD_MAX_CYCLES + 1, C.byref(nc)),
            "rrc_lowcad_schedule")
    return [(buf[c], buf[c + 1]) for c in range(nc.value)]


class LowCadence:
    """Low-cadence calibration of U units of an n x n grid (Sec. 4): the
    round-robin X-engine over each cycle's samples, then the omnical solve
    over every type (rrc_lowcad_*)."""

    def __init__(self, n: int, n_units: int, n_time: int, p: float = 1.0, log_base: float = 0.0,
                 one_cycle: bool = False):
        self._lib = L.load_library()
        self.n, self.n_units, self.n_time = n, n_units, n_time
        # one_cycle: every type in one cycle over the whole interval, i.e. the
        # full visibility matrix V^full of an FX correlator
        self.cycles = [(0, 2 * n * (n - 1))] if one_cycle else lowcad_schedule(n, p, log_base)
        flat = [c[0] for c in self.cycles] + [self.cycles[-1][1]]
        self._tb = (C.c_int32 * len(flat))(*flat)
        self.n_pairs = n * n * (n * n - 1) // 2
        self.n_types = 2 * n * (n - 1)

    def xengine(self, volt: torch.Tensor) -> torch.Tensor:
        shape = (self.n_units, self.n_time, self.n * self.n)
        if tuple(volt.shape) != shape or volt.dtype != torch.complex64 or not volt.is_cuda or not volt.is_contiguous():
            raise ValueError(f"volt must be a contiguous complex64 CUDA tensor of shape {shape}")
        out = torch.empty((self.n_units, self.n_pairs), dtype=torch.complex64, device=volt.device)
        L.check(self._lib.rrc_lowcad_xengine(self.n, self.n_units, self.n_time, self._tb, len(self.cycles),
                                             _stream(), _ptr(volt), _ptr(out)), "rrc_lowcad_xengine")
        return out

    def solve(self, vfull: torch.Tensor, gains_in: torch.Tensor, max_iter: int = 20000, tol: float = 1e-7):
        dev = vfull.device
        U = self.n_units
        if tuple(vfull.shape) != (U, self.n_pairs) or vfull.dtype != torch.complex64 or not vfull.is_contiguous():
            raise ValueError("vfull must be contiguous complex64 [U, N(N-1)/2]")
        if tuple(gains_in.shape) != (U, self.n * self.n) or gains_in.dtype != torch.complex64 \
                or not gains_in.is_contiguous():
            raise ValueError("gains_in must be contiguous complex64 [U, N]")
        out = dict(gains=torch.empty((U, self.n * self.n), dtype=torch.complex64, device=dev),
                   vmodel=torch.empty((U, self.n_types), dtype=torch.complex64, device=dev),
                   chisq=torch.empty((U,), dtype=torch.float32, device=dev),
                   niter=torch.zeros((U,), dtype=torch.int32, device=dev),
                   status=torch.empty((U,), dtype=torch.int32, device=dev))
        L.check(self._lib.rrc_lowcad_solve(self.n, U, _stream(), _ptr(vfull), _ptr(gains_in), int(max_iter),
                                           float(tol), _ptr(out["gains"]), _ptr(out["vmodel"]), _ptr(out["chisq"]),
                                           _ptr(out["niter"]), _ptr(out["status"])), "rrc_lowcad_solve")
        return out


def chisq_full(n: int, vfull: torch.Tensor, gains: torch.Tensor, vunique: torch.Tensor):
    """Whole-array fit of the FFT-correlator's model to the full visibility
    matrix (rrc_chisq_full): returns (chisq [U], chisq_cal [U]) float64."""
    lib = L.load_library()
    U = vfull.shape[0]
    N = n * n
    for t, shape, name in ((vfull, (U, N * (N - 1) // 2), "vfull"), (gains, (U, N), "gains"),
                           (vunique, (U, 2 * n * (n - 1)), "vunique")):
        if tuple(t.shape) != shape or t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous complex64 CUDA tensor of shape {shape}")
    c = torch.empty((U,), dtype=torch.float64, device=vfull.device)
    cc = torch.empty((U,), dtype=torch.float64, device=vfull.device)
    L.check(lib.rrc_chisq_full(n, U, _stream(), _ptr(vfull), _ptr(gains), _ptr(vunique), _ptr(c), _ptr(cc)),
            "rrc_chisq_full")
    return c, cc


def default_opts() -> Dict[str, float]:
    lib = L.load_library()
    o = L.SolverOpts()
    lib.rrc_default_opts(C.byref(o))
    return {f: getattr(o, f) for f, _ in L.SolverOpts._fields_}


class Plan:
    """A plan for U units (channels) of an n x n grid with T samples each;
    with `mask` (n*n bytes), of the antennas of a masked lattice such as a
    hexagonal array on its grid (rrc_plan_create_masked)."""

    def __init__(self, n: int, types: Sequence[Tuple[int, int]], n_units: int, n_time: int,
                 dtype: str = "c64", mask=None, **opts):
        self._lib = L.load_library()
        self.n = n
        self.types = [tuple(int(v) for v in t) for t in types]
        self.dtype = {"c64": L.RRC_C64, "ci4": L.RRC_CI4}[dtype]
        o = L.SolverOpts()
        self._lib.rrc_default_opts(C.byref(o))
        names = {"init_mode": {"firstcal": L.RRC_INIT_FIRSTCAL, "gains": L.RRC_INIT_GAINS},
                 "degen_mode": {"refant": L.RRC_DEGEN_REFANT, "match": L.RRC_DEGEN_MATCH}}
        for key, val in opts.items():
            if key in names and isinstance(val, str):
                val = names[key][val]
            setattr(o, key, val)
        self.opts = o
        h = C.c_void_p()
        if mask is None:
            L.check(self._lib.rrc_plan_create(C.byref(h), n, _types_array(self.types), len(self.types),
                                              n_units, n_time, self.dtype, C.byref(o)), "rrc_plan_create")
        else:
            m = _mask_arg(n, mask)
            L.check(self._lib.rrc_plan_create_masked(C.byref(h), n, m.ctypes.data, _types_array(self.types),
                                                     len(self.types), n_units, n_time, self.dtype, C.byref(o)),
                    "rrc_plan_create_masked")
        self._h = h
        info = L.PlanInfo()
        L.check(self._lib.rrc_plan_get_info(h, C.byref(info)), "rrc_plan_get_info")
        self.info = {f: getattr(info, f) for f, _ in L.PlanInfo._fields_}
        self.n_ant = info.n_ant
        self.n_pairs = info.n_pairs
        self.n_lags = info.n_lags
        self.n_units = n_units
        self.n_time = n_time
        self.dof = info.dof
        self._ws: Optional[torch.Tensor] = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.rrc_plan_destroy(h)
            self._h = None

    # ------------------------------------------------------------ helpers
    def workspace(self, device="cuda") -> torch.Tensor:
        nb = int(self.info["workspace_bytes"])
        if self._ws is None or self._ws.device != torch.device(device) or self._ws.numel() < nb:
            self._ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=device)
        return self._ws

    def _check_volt(self, volt: torch.Tensor):
        shape = (self.n_units, self.n_time, self.n_ant)
        want = torch.complex64 if self.dtype == L.RRC_C64 else torch.uint8
        if tuple(volt.shape) != shape or volt.dtype != want or not volt.is_cuda or not volt.is_contiguous():
            raise ValueError(f"volt must be a contiguous {want} CUDA tensor of shape {shape}, "
                             f"got {volt.dtype} {tuple(volt.shape)} on {volt.device}")

    def _check_c64(self, t: Optional[torch.Tensor], shape, name):
        if t is None:
            return
        if tuple(t.shape) != tuple(shape) or t.dtype != torch.complex64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous complex64 CUDA tensor of shape {tuple(shape)}")

    def vred_like(self, device) -> torch.Tensor:
        if self.dtype == L.RRC_CI4:
            return torch.empty((self.n_units, self.n_pairs, 2), dtype=torch.int32, device=device)
        return torch.empty((self.n_units, self.n_pairs), dtype=torch.complex64, device=device)

    # -------------------------------------------------------------- calls
    def fftcorr(self, volt: torch.Tensor, gains: torch.Tensor):
        """(a1)-(a3): returns (V^unique [U, n_lags] complex64, V_auto [U] float32)."""
        self._check_volt(volt)
        self._check_c64(gains, (self.n_units, self.n_ant), "gains")
        vu = torch.empty((self.n_units, self.n_lags), dtype=torch.complex64, device=volt.device)
        va = torch.empty((self.n_units,), dtype=torch.float32, device=volt.device)
        L.check(self._lib.rrc_fftcorr(self._h, _stream(), _ptr(volt), _ptr(gains), _ptr(vu), _ptr(va),
                                      _ptr(self.workspace(volt.device))), "rrc_fftcorr")
        return vu, va

    def xengine(self, volt: torch.Tensor) -> torch.Tensor:
        """(a4): V^reduced [U, P] complex64, or [U, P, 2] int32 raw sums for 4-bit data."""
        self._check_volt(volt)
        vr = self.vred_like(volt.device)
        L.check(self._lib.rrc_xengine(self._h, _stream(), _ptr(volt), _ptr(vr),
                                      _ptr(self.workspace(volt.device))), "rrc_xengine")
        return vr

    def solve(self, vred: torch.Tensor, gains_in: Optional[torch.Tensor] = None,
              gains_ref: Optional[torch.Tensor] = None) -> Dict[str, torch.Tensor]:
        """(a5): gains [U, N], vmodel [U, K], chisq [U], niter [U], status [U]."""
        dev = vred.device
        want = self.vred_like(dev)
        if tuple(vred.shape) != tuple(want.shape) or vred.dtype != want.dtype or not vred.is_contiguous():
            raise ValueError(f"vred must be contiguous {want.dtype} of shape {tuple(want.shape)}")
        self._check_c64(gains_in, (self.n_units, self.n_ant), "gains_in")
        self._check_c64(gains_ref, (self.n_units, self.n_ant), "gains_ref")
        out = dict(gains=torch.empty((self.n_units, self.n_ant), dtype=torch.complex64, device=dev),
                   vmodel=torch.empty((self.n_units, len(self.types)), dtype=torch.complex64, device=dev),
                   chisq=torch.empty((self.n_units,), dtype=torch.float32, device=dev),
                   niter=torch.empty((self.n_units,), dtype=torch.int32, device=dev),
                   status=torch.empty((self.n_units,), dtype=torch.int32, device=dev))
        L.check(self._lib.rrc_solve(self._h, _stream(), _ptr(vred), _ptr(gains_in), _ptr(gains_ref),
                                    _ptr(out["gains"]), _ptr(out["vmodel"]), _ptr(out["chisq"]),
                                    _ptr(out["niter"]), _ptr(out["status"]), _ptr(self.workspace(dev))),
                "rrc_solve")
        return out

    def omnical(self, vred: torch.Tensor, gains_in: Optional[torch.Tensor] = None, max_iter: int = 100000,
                tol: float = 1e-6, finish: bool = True, state: Optional[Dict[str, torch.Tensor]] = None):
        """(a5) omnical's damped updates (rrc_omnical): one call of up to
        max_iter iterations.  `state` (gains, vmodel, chisq, niter, status,
        delta) is created when None and carried between calls."""
        dev = vred.device
        want = self.vred_like(dev)
        if tuple(vred.shape) != tuple(want.shape) or vred.dtype != want.dtype or not vred.is_contiguous():
            raise ValueError(f"vred must be contiguous {want.dtype} of shape {tuple(want.shape)}")
        self._check_c64(gains_in, (self.n_units, self.n_ant), "gains_in")
        if state is None:
            if gains_in is None:
                raise ValueError("the first call needs gains_in")
            U = self.n_units
            state = dict(gains=torch.empty((U, self.n_ant), dtype=torch.complex64, device=dev),
                         vmodel=torch.empty((U, len(self.types)), dtype=torch.complex64, device=dev),
                         chisq=torch.zeros((U,), dtype=torch.float32, device=dev),
                         niter=torch.zeros((U,), dtype=torch.int32, device=dev),
                         status=torch.zeros((U,), dtype=torch.int32, device=dev),
                         delta=torch.zeros((U,), dtype=torch.float32, device=dev))
        L.check(self._lib.rrc_omnical(self._h, _stream(), _ptr(vred), _ptr(gains_in), int(max_iter), float(tol),
                                      1 if finish else 0, _ptr(state["gains"]), _ptr(state["vmodel"]),
                                      _ptr(state["chisq"]), _ptr(state["niter"]), _ptr(state["status"]),
                                      _ptr(state["delta"]), _ptr(self.workspace(dev))), "rrc_omnical")
        return state

    def chisq_fwd(self, g, vm, vred) -> torch.Tensor:
        self._check_c64(g, (self.n_units, self.n_ant), "g")
        self._check_c64(vm, (self.n_units, len(self.types)), "vm")
        self._check_c64(vred, (self.n_units, self.n_pairs), "vred")
        out = torch.empty((self.n_units,), dtype=torch.float32, device=g.device)
        L.check(self._lib.rrc_chisq_fwd(self._h, _stream(), _ptr(g), _ptr(vm), _ptr(vred), _ptr(out)),
                "rrc_chisq_fwd")
        return out

    def chisq_adj(self, g, vm, vred):
        """(a6): (2 dchi2/dconj(g), 2 dchi2/dconj(V), diag_g, diag_v)."""
        self._check_c64(g, (self.n_units, self.n_ant), "g")
        self._check_c64(vm, (self.n_units, len(self.types)), "vm")
        self._check_c64(vred, (self.n_units, self.n_pairs), "vred")
        gg = torch.empty_like(g)
        gv = torch.empty_like(vm)
        dg = torch.empty(g.shape, dtype=torch.float32, device=g.device)
        dv = torch.empty(vm.shape, dtype=torch.float32, device=g.device)
        L.check(self._lib.rrc_chisq_adj(self._h, _stream(), _ptr(g), _ptr(vm), _ptr(vred), _ptr(gg),
                                        _ptr(gv), _ptr(dg), _ptr(dv)), "rrc_chisq_adj")
        return gg, gv, dg, dv

    def run_io(self, volt: torch.Tensor, gains_in: Optional[torch.Tensor], gains_ref: Optional[torch.Tensor],
               out: Dict[str, torch.Tensor], work: Optional[torch.Tensor] = None) -> "L.RunIO":
        """The rrc_io of one run (argument checks and marshalling only).
        `out` may hold "stamps": [1 + U] int64 (device-clock stamps)."""
        self._check_volt(volt)
        self._check_c64(gains_in, (self.n_units, self.n_ant), "gains_in")
        self._check_c64(gains_ref, (self.n_units, self.n_ant), "gains_ref")
        st = out.get("stamps")
        if st is not None and (tuple(st.shape) != (1 + self.n_units,) or st.dtype != torch.int64
                               or not st.is_cuda or not st.is_contiguous()):
            raise ValueError(f"stamps must be a contiguous int64 CUDA tensor of shape ({1 + self.n_units},)")
        dev = volt.device
        if work is None:
            work = self.workspace(dev)
        return L.RunIO(_ptr(volt), _ptr(gains_in), _ptr(gains_ref), _ptr(out["vunique"]), _ptr(out["vauto"]),
                       _ptr(out["vred"]), _ptr(out["gains"]), _ptr(out["vmodel"]), _ptr(out["chisq"]),
                       _ptr(out["niter"]), _ptr(out["status"]), _ptr(work), _ptr(st))

    def run(self, volt: torch.Tensor, gains_in: Optional[torch.Tensor] = None,
            gains_ref: Optional[torch.Tensor] = None, mode: str = "pipelined",
            out: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        """The whole hot path (rrc_run); `out` may supply preallocated outputs."""
        if out is None:
            out = self.alloc_outputs(volt.device)
        io = self.run_io(volt, gains_in, gains_ref, out)
        L.check(self._lib.rrc_run(self._h, _stream(), _MODES[mode], C.byref(io)), "rrc_run")
        return out

    def run_static(self, volt: torch.Tensor, gains_in: Optional[torch.Tensor] = None,
                   gains_ref: Optional[torch.Tensor] = None, mode: str = "pipelined",
                   out: Optional[Dict[str, torch.Tensor]] = None) -> Dict[str, torch.Tensor]:
        """rrc_run_static: the whole hot path on the library's static scratch
        (no workspace); the plan must be prepared (see `prepare`)."""
        if out is None:
            out = self.alloc_outputs(volt.device)
        io = self.run_io(volt, gains_in, gains_ref, out, work=None)
        io.d_work = None
        L.check(self._lib.rrc_run_static(self._h, _stream(), _MODES[mode], C.byref(io)), "rrc_run_static")
        return out

    def tune(self, volt: torch.Tensor, gains_in: torch.Tensor, out: Optional[Dict[str, torch.Tensor]] = None,
             cache_path: Optional[str] = None) -> Dict[str, float]:
        """rrc_plan_tune: pick the fastest launch parameters of the pipelined
        run (FFT time chunk, branch order, 4-bit X-engine kernel, FFT size);
        `out` is overwritten.  Returns the choice."""
        if out is None:
            out = self.alloc_outputs(volt.device)
        io = self.run_io(volt, gains_in, None, out)
        t = L.Tune()
        L.check(self._lib.rrc_plan_tune(self._h, _stream(), C.byref(io),
                                        cache_path.encode() if cache_path else None, C.byref(t)), "rrc_plan_tune")
        return {f: getattr(t, f) for f, _ in L.Tune._fields_}

    def set_order(self, order: str) -> None:
        """Branch order of the pipelined run: "xeng_first", "fft_first" or "serial"."""
        code = {"xeng_first": L.RRC_ORDER_XENG_FIRST, "fft_first": L.RRC_ORDER_FFT_FIRST,
                "serial": L.RRC_ORDER_SERIAL}[order]
        L.check(self._lib.rrc_plan_set_order(self._h, code), "rrc_plan_set_order")

    def set_xengine(self, kind: str) -> None:
        """X-engine kernel of a 4-bit plan: "auto", "dot" or "mfma"."""
        code = {"auto": L.RRC_XENG_AUTO, "dot": L.RRC_XENG_DOT, "mfma": L.RRC_XENG_MFMA}[kind]
        L.check(self._lib.rrc_plan_set_xengine(self._h, code), "rrc_plan_set_xengine")

    def set_fft_size(self, m: int) -> None:
        """Padded FFT size of the FFT-correlator: the default power of two, or
        48 for grids with 2n - 1 <= 48 whose default is larger."""
        L.check(self._lib.rrc_plan_set_fft_size(self._h, int(m)), "rrc_plan_set_fft_size")
        info = L.PlanInfo()
        L.check(self._lib.rrc_plan_get_info(self._h, C.byref(info)), "rrc_plan_get_info")
        self.info = {f: getattr(info, f) for f, _ in L.PlanInfo._fields_}

    def prepare(self) -> None:
        """Bind the plan to the current device and make its device resources."""
        L.check(self._lib.rrc_plan_prepare(self._h), "rrc_plan_prepare")

    def alloc_outputs(self, device) -> Dict[str, torch.Tensor]:
        U = self.n_units
        return dict(vunique=torch.empty((U, self.n_lags), dtype=torch.complex64, device=device),
                    vauto=torch.empty((U,), dtype=torch.float32, device=device),
                    vred=self.vred_like(device),
                    gains=torch.empty((U, self.n_ant), dtype=torch.complex64, device=device),
                    vmodel=torch.empty((U, len(self.types)), dtype=torch.complex64, device=device),
                    chisq=torch.empty((U,), dtype=torch.float32, device=device),
                    niter=torch.empty((U,), dtype=torch.int32, device=device),
                    status=torch.empty((U,), dtype=torch.int32, device=device))


_MODES = {"pipelined": L.RRC_RUN_PIPELINED, "selfcal": L.RRC_RUN_SELFCAL}


class Batch:
    """Several plans (arrays of possibly different grids) run concurrently
    in one call (rrc_batch_run)."""

    def __init__(self, plans: Sequence[Plan], graph: bool = False):
        self._lib = L.load_library()
        self.plans = list(plans)           # kept alive for the batch's lifetime
        arr = (C.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = C.c_void_p()
        flags = L.RRC_BATCH_GRAPH if graph else 0
        L.check(self._lib.rrc_batch_create(C.byref(h), len(self.plans), arr, flags), "rrc_batch_create")
        self._h = h
        self._ios = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.rrc_batch_destroy(h)
            self._h = None

    def run(self, volts: Sequence[torch.Tensor], gains_in: Sequence[Optional[torch.Tensor]],
            outs: Sequence[Dict[str, torch.Tensor]], mode: str = "pipelined",
            gains_ref: Optional[Sequence[Optional[torch.Tensor]]] = None) -> Sequence[Dict[str, torch.Tensor]]:
        if gains_ref is None:
            gains_ref = [None] * len(self.plans)
        if not (len(volts) == len(gains_in) == len(outs) == len(gains_ref) == len(self.plans)):
            raise ValueError("one voltage, gains and output set per plan")
        ios = (L.RunIO * len(self.plans))(*[p.run_io(v, gi, gr, o) for p, v, gi, gr, o
                                            in zip(self.plans, volts, gains_in, gains_ref, outs)])
        L.check(self._lib.rrc_batch_run(self._h, _stream(), _MODES[mode], ios), "rrc_batch_run")
        self._ios = ios
        return outs


def wall_clock_hz() -> float:
    """Ticks per second of the device clock that run stamps count."""
    lib = L.load_library()
    hz = C.c_double()
    L.check(lib.rrc_wall_clock_hz(C.byref(hz)), "rrc_wall_clock_hz")
    return hz.value


class ChiSq(torch.autograd.Function):
    """chi^2 per unit with the hand-written adjoint as its backward.

    backward returns grad_out * 2 dchi2/dconj(z), PyTorch's convention for
    the gradient of a real function of complex inputs.
    """

    @staticmethod
    def forward(ctx, g, vm, vred, plan):
        ctx.plan = plan
        ctx.save_for_backward(g, vm, vred)
        return plan.chisq_fwd(g.detach().contiguous(), vm.detach().contiguous(), vred.detach().contiguous())

    @staticmethod
    def backward(ctx, grad_out):
        g, vm, vred = ctx.saved_tensors
        gg, gv, _, _ = ctx.plan.chisq_adj(g.detach().contiguous(), vm.detach().contiguous(),
                                          vred.detach().contiguous())
        go = grad_out.to(torch.float32)
        return gg * go[:, None], gv * go[:, None], None, None


def chisq(g: torch.Tensor, vm: torch.Tensor, vred: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable chi^2 (per unit) of eq. redchi with uniform noise."""
    return ChiSq.apply(g, vm, vred, plan)
