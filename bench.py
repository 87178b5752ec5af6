"""Throughput of the calibrated FFT-correlator on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
    python bench.py --copy-calibration      # the HBM-counter calibration copy

One step = one integration of every unit (array, channel) of the workload
through the whole hot path: reduced X-engine, FFT-correlator (gain
application, padded spatial FFT, |.|^2 integration, inverse transform and
redundant normalisation) and the reduced redundant calibration solve.  The
batched path issues the step for all units at once (rrc_run, PIPELINED: the
FFT applies the previous integration's gains; several arrays run together on
branch streams through rrc_batch_run); the plain path calibrates one
channel at a time, synchronising after each.  Inputs are resident in HBM
before timing starts.  Prints one JSON line.

The default workload is the 64x64-grid, 1024-channel, 4096-sample 4-bit one
(the largest single-GPU configuration); the 32x32-grid, 256-channel
complex64 one and the paper's 331-antenna hexagonal array (1024 channels,
2048 samples) are measured beside it under "extra".
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg: str) -> None:
    """Progress of the run on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)

# 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz; the 157.3 TFLOP/s
# vector figure counts packed (two-wide) FP32, which these kernels do not use
VALU_FP32_PEAK_TFLOPS = 78.6
METRIC = "calibrated channel-integrations/sec (batched+adjoint vs plain) at stated gain error"
DEFAULT_WORKLOAD = "g64_c1024_t4096_ci4"
EXTRA_WORKLOAD = "g32_c256_t2048"


def pad_size(n: int) -> int:
    """The plan's default FFT size: the smallest of 16, 32, 48, 64, 96, 128
    with M >= 2n - 1."""
    return min(m for m in (16, 32, 48, 64, 96, 128) if m >= 2 * n - 1)


def fft_flops_per_sample(n: int, m: int = 0) -> float:
    """Algorithmic FP32 flops of one sample's FFT-correlator work.

    The practical count of the hot-path scope: every row (n of them) and
    column (M) transform of the padded M-point FFT costs 4.25 M log2 M flops
    less its first (trivial, half-zero) stage, i.e. 4.25 M (log2 M - 1);
    |E|^2 accumulation 4 flops per grid point; gain application 6 flops per
    antenna.  M is the plan's FFT size (by default the smallest with
    M >= 2n - 1): at n = 16, 32, 64 this gives 32.5 MF, 314 MF and 2.94 GF
    per unit of 1024, 2048 and 4096 samples.  The mixed-radix sizes count
    the transforms the kernels run.
    """
    m = m or pad_size(n)
    if m == 48:
        # two 24-point halves, each a radix-3 step (8 butterflies of 30
        # flops) and three 8-point radix-2^2 transforms
        per = 2 * (8 * 30 + 3 * 4.25 * 8 * 3)
    elif m == 96:
        # three 32-point transforms and their folded inputs: a twiddle on
        # each of the 96 inputs, a partner term on 16 per third
        per = 3 * 4.25 * 32 * 5 + 3 * 32 * 6 + 3 * 16 * 8
    else:
        per = 4.25 * m * (math.log2(m) - 1)
    return (n + m) * per + 4 * m * m + 6 * n * n


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the second (32x32) workload")
    ap.add_argument("--gate-units", type=int, default=8)
    ap.add_argument("--plain-units", type=int, default=0,
                    help="channels timed in the plain per-channel form (0: up to 256, within 20 s)")
    ap.add_argument("--inflight", type=int, default=0,
                    help="batches in flight: step i runs on lane i mod D, each lane with its own "
                         "stream, plans, input copy and outputs; 0 picks enough for the solves "
                         "(one workgroup per unit) of all lanes to cover the CUs, at most 4")
    ap.add_argument("--order", default="auto", choices=["auto", "xeng_first", "fft_first", "serial"],
                    help="pipelined branch order (auto: serial for 4-bit workloads, whose VALU-bound "
                         "FFT stage and solve each fill the device and slow each other down when they "
                         "share it; X-engine first otherwise)")
    ap.add_argument("--latency-reps", type=int, default=50)
    ap.add_argument("--xengine", default="auto", choices=["auto", "dot", "mfma"],
                    help="X-engine kernel of 4-bit plans (auto: the dot-product kernel)")
    ap.add_argument("--stages-only", action="store_true",
                    help="only time each stage alone (--steps launches each; the profiling run whose "
                         "kernel averages are the stage times of the roofline) and print them")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB three times (the run whose FETCH_SIZE / WRITE_SIZE scale "
                         "the HBM counters of the kernels)")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = 256 * 1024 * 1024 // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copied 3 x", n * 4, "bytes", flush=True)


def measured_traffic(workload: str):
    """HBM bytes per launch of the FFT-correlator stage from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by a copy of known size),
    or None when none was taken for this workload or the kernels' sources
    have changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_fftcorr_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    for src, h in d["sources_sha1"].items():
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha1(f.read()).hexdigest() != h:
                return None
    return d["hbm_bytes_per_launch"]


# --------------------------------------------------------------- the GPU run

def setup(w, dev, rrc, inflight, order, xengine="auto"):
    import torch
    from synthdata import workload_voltages
    from synthdata.device import device_voltages
    dtype = "ci4" if w.ci4 else "c64"
    # small workloads: the host generator's exact bytes; large: drawn on the GPU
    host_gen = len(w.grids) == 1 and w.grids[0] ** 2 * w.n_chan * w.n_time <= 64 * 1024 * 1024
    rng = np.random.default_rng(7)
    arrays = []
    for ai, n in enumerate(w.grids):
        if host_gen:
            vnp, g = workload_voltages(w, ai)
            volt = torch.from_numpy(vnp).to(dev)
        else:
            volt, g = device_voltages(w, ai, dev)
        types, npairs = rrc.select_subset(n)
        arrays.append(dict(name=f"g{n}", ai=ai, n=n, types=types, npairs=npairs, volt=volt, gains_host=g,
                           gains_in=torch.from_numpy(g.astype(np.complex64)).to(dev),
                           sample=rng.permutation(w.n_chan).tolist()))
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    D = inflight if inflight > 0 else max(1, min(4, -(-cus // (w.n_chan * len(arrays)))))
    if order == "auto":
        order = "serial" if w.ci4 else "xeng_first"
    lanes = []
    for li in range(D):
        la = []
        for a in arrays:
            plan = rrc.Plan(a["n"], a["types"], w.n_chan, w.n_time, dtype=dtype)
            plan.set_order(order)
            if w.ci4:
                plan.set_xengine(xengine)
            plan.workspace(dev)            # allocated here, not in a timed step
            la.append(dict(a, plan=plan, out=plan.alloc_outputs(dev),
                           volt=a["volt"] if li == 0 else a["volt"].clone(),
                           gains_in=a["gains_in"] if li == 0 else a["gains_in"].clone()))
        lanes.append(dict(arrays=la, stream=torch.cuda.Stream(dev),
                          batch=rrc.Batch([a["plan"] for a in la]) if len(la) > 1 else None))
    torch.cuda.synchronize()
    return dict(arrays=lanes[0]["arrays"], lanes=lanes, D=D, cus=cus, dtype=dtype, host_gen=host_gen,
                order=order)


def run_lane(ln):
    if ln["batch"] is None:
        a = ln["arrays"][0]
        a["plan"].run(a["volt"], gains_in=a["gains_in"], mode="pipelined", out=a["out"])
    else:
        la = ln["arrays"]
        ln["batch"].run([a["volt"] for a in la], [a["gains_in"] for a in la], [a["out"] for a in la],
                        mode="pipelined")


def time_steps(S, steps, warmup):
    """W untimed steps, then K steps between HIP events on the launch
    stream (every lane waits for the start event; the launch stream waits
    for every lane before the end event); synchronised on both sides."""
    import torch
    lanes, D = S["lanes"], S["D"]
    stream = torch.cuda.current_stream()

    def step(i):
        ln = lanes[i % D]
        with torch.cuda.stream(ln["stream"]):
            run_lane(ln)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for ln in lanes:
        ln["stream"].wait_event(e0)
    for i in range(steps):
        step(i)
    for ln in lanes:
        stream.wait_stream(ln["stream"])
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_fn(fn, reps):
    """Average time per call of fn, HIP events on the current stream."""
    import torch
    stream = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a_.record(stream)
    for _ in range(reps):
        fn()
    b_.record(stream)
    torch.cuda.synchronize()
    return a_.elapsed_time(b_) / reps


def stage_times(S, w, reps):
    """Each stage alone, per launch (all channels of an array), summed over
    arrays; the solve is timed on the X-engine's output."""
    st = {"xengine": 0.0, "fftcorr": 0.0, "solve": 0.0}
    for a in S["arrays"]:
        p = a["plan"]
        vred = []
        st["xengine"] += time_fn(lambda: vred.append(p.xengine(a["volt"])) if not vred else p.xengine(a["volt"]), reps)
        st["fftcorr"] += time_fn(lambda: p.fftcorr(a["volt"], a["gains_in"]), reps)
        st["solve"] += time_fn(lambda: p.solve(vred[0]), reps)
    return st


def latency_from_stamps(S, reps):
    """Per-array latency of the batched step from the device's own stamps:
    for each array, the time from its run's start on the device until the
    last of its units' outputs is written; p50 / p99 over `reps` steps."""
    import torch
    import paper_2005_03060_amd as rrc
    ln = S["lanes"][0]
    for a in ln["arrays"]:
        a["out"]["stamps"] = torch.zeros(1 + a["plan"].n_units, dtype=torch.int64, device=a["volt"].device)
    hz = rrc.wall_clock_hz()
    lat = {a["name"]: [] for a in ln["arrays"]}
    first = []
    for _ in range(reps):
        run_lane(ln)
        torch.cuda.synchronize()
        t0 = min(int(a["out"]["stamps"][0]) for a in ln["arrays"])
        first.append(t0)
        for a in ln["arrays"]:
            s = a["out"]["stamps"].cpu().numpy()
            lat[a["name"]].append((int(s[1:].max()) - t0) / hz * 1e3)
    for a in ln["arrays"]:
        a["out"].pop("stamps")
    return {k: {"p50_ms": float(np.percentile(v, 50)), "p99_ms": float(np.percentile(v, 99)),
                "reps": len(v), "source": "device wall-clock stamps (rrc_io.d_stamps)"} for k, v in lat.items()}


OMNI_TOL = 1e-6          # FP32 relative change at which omnical stops
OMNI_MAX_ITER = 20000


def plain_per_channel(S, w, rrc, dev, max_units, budget_s=20.0):
    """The plain form: one channel at a time, the paper's solver stepped from
    the host.  Per channel: the X-engine, omnical's damped updates one
    iteration per launch with the relative change read back after each
    (the per-iteration convergence check), the finishing launch, then the
    FFT-correlator, with a host synchronisation at the end.  Time per
    channel on the first channels (at most `max_units` or 256, and within
    the budget), scaled to all channels."""
    import torch
    per_array, timed, iters = [], [], []
    for a in S["arrays"]:
        p1 = rrc.Plan(a["n"], a["types"], 1, w.n_time, dtype=S["dtype"])
        nc = min(w.n_chan, 256 if max_units <= 0 else max_units)
        t_all, done = 0.0, 0
        for c in range(nc):
            v = a["volt"][c:c + 1]
            gi = a["gains_in"][c:c + 1]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            vr = p1.xengine(v)
            st = p1.omnical(vr, gains_in=gi, max_iter=1, tol=OMNI_TOL, finish=False)
            it = 1
            while float(st["delta"][0]) >= OMNI_TOL and it < OMNI_MAX_ITER:
                st = p1.omnical(vr, max_iter=1, tol=OMNI_TOL, finish=False, state=st)
                it += 1
            p1.omnical(vr, max_iter=0, tol=OMNI_TOL, finish=True, state=st)
            p1.fftcorr(v, gi)
            torch.cuda.synchronize()
            t_all += time.perf_counter() - t0
            done += 1
            iters.append(it)
            if t_all > budget_s / len(S["arrays"]):
                break
        per_array.append(t_all / done * w.n_chan)
        timed.append(done)
    return sum(per_array) * 1e3, timed, float(np.mean(iters))


def batched_omnical(S, w):
    """omnical on every unit of each array in one launch (device-side
    convergence): the solver alone, beside the Gauss-Newton solve's stage
    time.  Returns (ms, mean iterations, converged units)."""
    import torch
    ms, its, conv = 0.0, [], 0
    for a in S["arrays"]:
        p = a["plan"]
        vr = p.xengine(a["volt"])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        st = p.omnical(vr, gains_in=a["gains_in"], max_iter=OMNI_MAX_ITER, tol=OMNI_TOL, finish=True)
        e1.record()
        torch.cuda.synchronize()
        ms += e0.elapsed_time(e1)
        its += st["niter"].cpu().tolist()
        conv += int((st["status"] == 0).sum())
    return ms, float(np.mean(its)), conv


# ------------------------------------------------------------- oracle legs

def unpack(volt_u):
    from synthdata import unpack_ci4
    re, im = unpack_ci4(volt_u)
    return re, im


def gate_units(S, w, n_units):
    """Accuracy gate on seeded units: V^reduced (bit for bit for 4-bit data,
    else against the FP64 X-engine), the solved gains against the oracle's
    solve of the oracle's own V^reduced (identical integers for 4-bit data,
    FP64 sums for float), V^unique against eq. modelvis with the gains the
    FFT applied (every lag up to 32x32 grids; sampled lags from exact
    integer correlations beyond)."""
    from oracle import correlator as OC
    from oracle import geometry as OG
    from oracle import redcal as OR
    rep = {"units": [], "vred_bit_exact": None, "vred_max_rel": 0.0, "gains_max_rel": 0.0,
           "vunique_max_rel_l2": 0.0, "vunique_sampled_lag_max": None, "tol_gains": 1e-6,
           "tol_vunique": 1e-5, "status_nonzero": 0}
    per = max(1, n_units // len(S["arrays"]))
    exact = True
    for a in S["arrays"]:
        n, types = a["n"], a["types"]
        pos = OG.square_positions(n)
        idx = OG.PositionIndex(pos)
        pairs, tix = OG.group_pairs(pos, types)
        lags = OC.canonical_lags(n)
        out = a["out"]
        rep["status_nonzero"] += int((out["status"] != 0).sum())
        for u in a["sample"][:per]:
            g_in = a["gains_in"][u].cpu().numpy().astype(np.complex128)
            vr_gpu = out["vred"][u].cpu().numpy()
            if S["dtype"] == "ci4":
                re, im = unpack(a["volt"][u].cpu().numpy())
                sums = OC.xengine_int(re, im, pairs)
                exact &= bool(np.array_equal(vr_gpu.astype(np.int64), sums))
                vref = sums[:, 0] + 1j * sums[:, 1]
                # V^unique at sampled lags from exact integer correlations
                N, T = n * n, w.n_time
                rng = np.random.default_rng(u)
                pick = sorted(set([0, 1, n - 1, n, 2 * n]) | set(rng.choice(len(lags), 11, replace=False).tolist()))
                sel = [lags[k] for k in pick]
                vfull = np.zeros((N, N), dtype=np.complex128)
                for dx, dy in sel:
                    i, j = idx.pairs_of(dx, dy)
                    s = OC.xengine_int(re, im, np.stack([i, j], axis=1))
                    vfull[i, j] = (s[:, 0] + 1j * s[:, 1]) / T
                d = np.arange(N)
                s = OC.xengine_int(re, im, np.stack([d, d], axis=1))
                vfull[d, d] = s[:, 0] / T
                ref = OC.redundant_average(vfull, g_in, pos, sel)
                aref = OC.calibrated_auto(vfull, g_in)
                got = out["vunique"][u].cpu().numpy()[pick]
                nd = np.array([len(idx.pairs_of(dx, dy)[0]) for dx, dy in sel])
                # error uniform in the un-normalised correlation N_d T V(d)
                errn = float(np.max(np.abs(got - ref) * nd / (N * aref)))
                rep["vunique_sampled_lag_max"] = max(rep["vunique_sampled_lag_max"] or 0.0, errn)
                short = [k for k, (dx, dy) in enumerate(sel) if abs(dx) + dy <= 2]
                e = float(np.linalg.norm(got[short] - ref[short]) / np.linalg.norm(ref[short]))
                rep["vunique_max_rel_l2"] = max(rep["vunique_max_rel_l2"], e)
            else:
                v = a["volt"][u].cpu().numpy().astype(np.complex128)
                vf = OC.fx_correlate(v)
                vref = OC.xengine(vf, pairs)
                sc = np.mean(np.abs(v) ** 2)
                rep["vred_max_rel"] = max(rep["vred_max_rel"], float(np.max(np.abs(vr_gpu - vref)) / sc))
                ref = OC.redundant_average(vf, g_in, pos, lags)
                e = float(np.linalg.norm(out["vunique"][u].cpu().numpy() - ref) / np.linalg.norm(ref))
                rep["vunique_max_rel_l2"] = max(rep["vunique_max_rel_l2"], e)
            sol = OR.calibrate(vref, pos, types, pairs, tix)
            g = out["gains"][u].cpu().numpy().astype(np.complex128)
            rep["gains_max_rel"] = max(rep["gains_max_rel"], float(np.max(np.abs(g - sol["g"]) / np.abs(sol["g"]))))
            rep["units"].append(f"{a['name']}:{u}")
            log(f"gate unit {a['name']}:{u} done")
    if S["dtype"] == "ci4":
        rep["vred_bit_exact"] = exact
        rep.pop("vred_max_rel")
    else:
        rep["tol_gains"] = 1e-4      # whole float path: FP32 X-engine, then the solve
        rep.pop("vunique_sampled_lag_max")
    rep["n_units"] = len(rep["units"])
    return rep


def cpu_baseline(S, w, budget_s):
    """The FP64 oracle as it stands on a bounded sample of the same units:
    FX correlator (zgemm), X-engine, FIRSTCAL + Gauss-Newton to 1e-10,
    degeneracy fix, eq. modelvis average over every lag.  Whole units, one
    at a time, until at least min(10 s, budget) of work; at 4096 antennas a
    unit alone takes longer, so one unit is run.  Also a one-thread figure:
    the same unit with BLAS limited to one thread, its FX correlation timed
    on 1/16 of the samples and scaled by 16 (zgemm cost is linear in T)."""
    import threadpoolctl
    from oracle import correlator as OC
    from oracle import geometry as OG
    from oracle import redcal as OR
    a = S["arrays"][-1]
    n, types = a["n"], a["types"]
    pos = OG.square_positions(n)
    pairs, tix = OG.group_pairs(pos, types)
    lags = OC.canonical_lags(n)

    def volt64(u):
        vv = a["volt"][u].cpu().numpy()
        if vv.dtype == np.uint8:
            re, im = unpack(vv)
            return re.astype(np.float64) + 1j * im.astype(np.float64)
        return vv.astype(np.complex128)

    def one_unit(v, t_fx_scale=1):
        t = time.perf_counter()
        vf = OC.fx_correlate(v)
        t_fx = (time.perf_counter() - t) * t_fx_scale
        t = time.perf_counter()
        vred = OC.xengine(vf, pairs)
        cal = OR.calibrate(vred, pos, types, pairs, tix)
        OC.redundant_average(vf, cal["g"], pos, lags)
        return t_fx + (time.perf_counter() - t)

    done, t_all = 0, 0.0
    min_s = min(10.0, budget_s)
    for u in a["sample"]:
        t_all += one_unit(volt64(u))
        done += 1
        if t_all >= min_s or t_all * (done + 1) / done > budget_s:
            break
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    v = volt64(a["sample"][0])
    with threadpoolctl.threadpool_limits(1):
        t1 = one_unit(v[: max(1, v.shape[0] // 16)], t_fx_scale=16)
    return {"value": done / t_all, "unit": "calibrated channel-integrations/s", "cores": threads,
            "kind": "oracle", "os_cpu_count": os.cpu_count(),
            "one_thread_value": 1.0 / t1,
            "sample": f"{done} whole unit(s) of array {a['name']} of {w.name}, one at a time ({t_all:.1f} s, "
                      f"BLAS on {threads} threads): FX correlator (zgemm), X-engine gather, FIRSTCAL + "
                      f"Gauss-Newton to 1e-10, degeneracy fix, eq. modelvis average; one-thread figure: one "
                      f"unit, FX correlation on 1/16 of the samples scaled by 16"}


# ------------------------------------------------------------------ record

def measure(w, args, rrc, dev, with_oracle):
    log(f"{w.name}: generating inputs")
    S = setup(w, dev, rrc, args.inflight, args.order, args.xengine)
    if args.stages_only:
        log(f"{w.name}: stage times ({args.steps} launches each)")
        return {"stages_ms": stage_times(S, w, args.steps), "config": {"workload": w.name,
                                                                       "xengine": args.xengine}}
    log(f"{w.name}: {args.warmup} warm-up + {args.steps} timed steps")
    ms = time_steps(S, args.steps, args.warmup)
    log(f"{w.name}: {ms:.3f} ms per step; stage times")
    total_units = w.n_chan * len(S["arrays"])
    import torch
    serial_ms = time_fn(lambda: run_lane(S["lanes"][0]), args.steps)
    stages = stage_times(S, w, max(3, min(args.steps, 20)))
    flops = sum(fft_flops_per_sample(a["n"], a["plan"].info["fft_size"]) * w.n_time * w.n_chan for a in S["arrays"])
    vbytes = sum((1.0 if w.ci4 else 8.0) * a["n"] ** 2 * w.n_time * w.n_chan for a in S["arrays"])
    fft_s = stages["fftcorr"] * 1e-3
    x_s = stages["xengine"] * 1e-3
    tf = flops / fft_s / 1e12
    gbs = vbytes / fft_s / 1e9
    # the roof that binds: flop/B of the stage against the ridge of the
    # non-packed FP32 VALU and HBM peaks (9.8 flop/B)
    alu = flops / vbytes > VALU_FP32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    kernel = "FFT-correlator stage (k_fftcorr_q + k_fftfin)" if max(a["n"] for a in S["arrays"]) > 32 else \
        "FFT-correlator stage (k_fftcorr + k_fftfin_fft)"
    traffic = measured_traffic(w.name) if len(S["arrays"]) == 1 else None
    if alu:
        roof = {"bound": "alu", "achieved": tf, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / VALU_FP32_PEAK_TFLOPS, "traffic": traffic}
    else:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": traffic}
    roof.update({"kernel": kernel, "ms_per_launch": stages["fftcorr"], "units_per_launch": total_units,
                 "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": vbytes,
                 "hbm_achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                 "valu_achieved_TFLOPs": tf, "valu_frac": tf / VALU_FP32_PEAK_TFLOPS})
    other = [
        {"kernel": "k_xant + k_xfin (reduced X-engine)", "bound": "hbm", "ms_per_launch": stages["xengine"],
         "achieved": vbytes / x_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": vbytes / x_s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": vbytes},
        {"kernel": "k_solve (reduced redundant calibration)", "bound": "latency",
         "ms_per_launch": stages["solve"], "units_per_launch": total_units, "workgroups_per_unit": 1,
         "cus": S["cus"]},
    ]
    log(f"{w.name}: plain per-channel form (host-stepped omnical)")
    plain_ms, plain_n, plain_it = plain_per_channel(S, w, rrc, dev, args.plain_units)
    log(f"{w.name}: batched omnical")
    om_ms, om_it, om_conv = batched_omnical(S, w)
    gn_it = float(np.mean(np.concatenate([a["out"]["niter"].cpu().numpy() for a in S["arrays"]])))
    rec = {
        "value": total_units / (ms * 1e-3), "ms_per_step": ms,
        "config": {"workload": w.name, "grids": [f"{a['n']}x{a['n']}" for a in S["arrays"]],
                   "antennas": [a["n"] ** 2 for a in S["arrays"]], "channels": w.n_chan, "samples": w.n_time,
                   "voltage_format": "ci4" if w.ci4 else "complex64",
                   "fft_size": [a["plan"].info["fft_size"] for a in S["arrays"]],
                   "types": [len(a["types"]) for a in S["arrays"]], "pairs": [a["npairs"] for a in S["arrays"]],
                   "mode": "pipelined, all channels per launch" +
                           (", arrays concurrently on branch streams" if len(S["arrays"]) > 1 else ""),
                   "branch_order": S["order"], "batches_in_flight": S["D"], "parallelism": "none (1 GPU)"},
        "stages_ms": stages,
        "one_batch_at_a_time": {"ms_per_step": serial_ms, "value": total_units / (serial_ms * 1e-3)},
        "plain_per_channel": {"ms_per_step": plain_ms, "value": total_units / (plain_ms * 1e-3),
                              "speedup_batched": plain_ms / ms, "channels_timed_per_array": plain_n,
                              "omnical_iterations_mean": plain_it, "omnical_tol": OMNI_TOL,
                              "form": "one channel at a time: X-engine, omnical (damping 0.3) one iteration "
                                      "per launch with the change read back after each, FFT-correlator; "
                                      "time per channel scaled to all channels"},
        "solver_comparison": {"gauss_newton_batched_ms": stages["solve"],
                              "gauss_newton_steps_mean": gn_it, "gauss_newton_start": "FIRSTCAL",
                              "omnical_batched_ms": om_ms, "omnical_iterations_mean": om_it,
                              "omnical_converged_units": om_conv, "omnical_start": "the given gains",
                              "units": total_units},
        "roofline": roof,
        "roofline_other": other,
        "data": "synthetic" + ("" if S["host_gen"] else " (drawn on the GPU)"),
    }
    if len(S["arrays"]) > 1:
        rec["per_array_latency"] = latency_from_stamps(S, args.latency_reps)
    if with_oracle:
        log(f"{w.name}: oracle gate on {args.gate_units} units")
        rec["gate"] = gate_units(S, w, args.gate_units)
        log(f"{w.name}: oracle timing")
        rec["cpu_baseline"] = cpu_baseline(S, w, 30.0)
    for ln in S["lanes"]:
        for a in ln["arrays"]:
            del a["volt"]
    del S
    torch.cuda.empty_cache()
    return rec


def measure_hex(side, n_chan, n_time, args, rrc, dev):
    """A hexagonal array (Sec. 3, Fig. 2) on its lattice grid: the whole
    path (rrc_run PIPELINED, the solve started from the given gains) over
    every channel, and each stage alone.  The 11-antennas-per-side hexagon is
    the paper's 331-antenna array (Sec. 6.4)."""
    import torch
    from synthdata import Workload
    from synthdata.device import device_voltages
    n, mask = rrc.hex_mask(side)
    w = Workload(5, f"hex{side}_c{n_chan}_t{n_time}", (n,), n_chan, n_time, 10.0,
                 note=f"hexagon of side {side} on its {n}x{n} grid")
    volt, g = device_voltages(w, 0, dev)
    types, npairs = rrc.select_subset_masked(n, mask, "hex")
    plan = rrc.Plan(n, types, n_chan, n_time, mask=mask, init_mode="gains")
    m = plan.info["fft_size"]
    plan.workspace(dev)
    gin = torch.from_numpy(g.astype(np.complex64)).to(dev)
    out = plan.alloc_outputs(dev)
    log(f"{w.name}: {args.warmup} warm-up + {args.steps} timed steps")
    ms = time_fn(lambda: plan.run(volt, gains_in=gin, mode="pipelined", out=out), max(args.steps, 20))
    st = {"xengine": time_fn(lambda: plan.xengine(volt), 10),
          "fftcorr": time_fn(lambda: plan.fftcorr(volt, gin), 10)}
    vred = plan.xengine(volt)
    st["solve"] = time_fn(lambda: plan.solve(vred, gains_in=gin), 10)
    torch.cuda.synchronize()
    flops = fft_flops_per_sample(n, m) * n_time * n_chan
    tf = flops / (st["fftcorr"] * 1e-3) / 1e12
    vbytes = 8.0 * n * n * n_time * n_chan
    status = int((out["status"] != 0).sum())
    del volt
    torch.cuda.empty_cache()
    return {"value": n_chan / (ms * 1e-3), "ms_per_step": ms,
            "config": {"workload": w.name, "layout": "hexagonal", "side": side, "grid": n,
                       "antennas": int(mask.sum()), "channels": n_chan, "samples": n_time,
                       "voltage_format": "complex64", "fft_size": m, "types": len(types),
                       "pairs": npairs, "mode": "pipelined, all channels per launch, solve from the given gains"},
            "stages_ms": st, "status_nonzero": status,
            "roofline": {"bound": "alu", "achieved": tf, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / VALU_FP32_PEAK_TFLOPS, "kernel": "FFT-correlator stage",
                         "algorithmic_flops_per_launch": flops, "hbm_frac": vbytes / (st["fftcorr"] * 1e-3) / 1e9 / HBM_PEAK_GBS}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); units shard across GPUs "
              f"with no collective, so the per-GPU figure is the one to scale.", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch
    import paper_2005_03060_amd as rrc
    from synthdata import WORKLOADS

    wl = {x.name: x for x in WORKLOADS}
    w = wl[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    r = measure(w, args, rrc, dev, with_oracle=not args.no_cpu_baseline)
    if args.stages_only:
        print(json.dumps(r), flush=True)
        return
    rec = {
        "metric": METRIC,
        "value": r["value"], "unit": "channel-integrations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": r["data"], "config": r["config"],
        "stages_ms": r["stages_ms"], "one_batch_at_a_time": r["one_batch_at_a_time"],
        "plain_per_channel": r["plain_per_channel"], "solver_comparison": r["solver_comparison"],
        "roofline": r["roofline"],
        "roofline_other": r["roofline_other"],
        "gate": r.get("gate"), "cpu_baseline": r.get("cpu_baseline"),
    }
    if "per_array_latency" in r:
        rec["per_array_latency"] = r["per_array_latency"]
    if args.workload == DEFAULT_WORKLOAD and not args.no_extra:
        a2 = argparse.Namespace(**vars(args))
        a2.steps = max(args.steps, 20)
        a2.gate_units = min(args.gate_units, 8)
        x = measure(wl[EXTRA_WORKLOAD], a2, rrc, dev, with_oracle=False)
        rec["extra"] = {EXTRA_WORKLOAD: {k: x[k] for k in ("value", "ms_per_step", "config", "stages_ms",
                                                           "roofline", "roofline_other", "plain_per_channel",
                                                           "solver_comparison")}}
        hx = measure_hex(11, 1024, 2048, a2, rrc, dev)
        rec["extra"][hx["config"]["workload"]] = hx
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
