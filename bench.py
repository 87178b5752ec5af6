"""Throughput of the calibrated FFT-correlator on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

One step = one integration of every unit (array, channel) of the workload
through the whole hot path: reduced X-engine, FFT-correlator (gain
application, padded spatial FFT, |.|^2 integration, inverse transform and
redundant normalisation) and the reduced redundant calibration solve.  The
batched path issues the steps for all units at once (rrc_run, PIPELINED: the
FFT applies the previous integration's gains; several arrays run together
through rrc_batch_run); the plain path calibrates one channel at a time,
synchronising after each.  Inputs are resident in HBM before timing starts.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_FP32_PEAK_TFLOPS = 78.6    # 256 CU x 64 lanes x 2 flop x 2.4 GHz, packed FP32 disabled
METRIC = "calibrated channel-integrations/sec (batched+adjoint vs plain) at stated gain error"


def fft_flops_per_sample(n: int, m: int) -> float:
    """Algorithmic FP32 flops of one sample's FFT-correlator work.

    Every row (n of them) and column (m) transform is an m-point FFT with
    only n <= m/2 non-zero inputs, done as two m/2-point FFTs
    (5 (m/2) log2(m/2) flops each) plus a pre-twiddle (6 flops per input)
    for the odd half; |E|^2 accumulation is 3 flops per grid point and the
    gain application 6 flops per antenna.
    """
    half = m // 2
    per_tf = 2 * 5 * half * np.log2(half) + 6 * half
    return (n + m) * per_tf + 3 * m * m + 6 * n * n


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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="g16_c64_t1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--inflight", type=int, default=0,
                    help="batches in flight: step i runs on lane i mod D, each lane with its own "
                         "stream, plans, input copy and outputs; 0 picks enough for the solves "
                         "(one workgroup per unit) of all lanes to cover the CUs, at most 4")
    return ap.parse_args()


def cpu_baseline(arrays, budget_s, gate_units):
    """The FP64 oracle, as it stands, on a bounded sample of the same units.

    Units are taken in a seeded random order, in passes over the sample,
    until at least min(10 s, budget) of oracle work is done, and never past
    the budget.  Also the accuracy gate: for the first `gate_units` of them the
    oracle solves the GPU's own V^reduced and the GPU gains are compared
    after the same degeneracy fix.  Arrays whose dense oracle solve is too
    slow for a bench (n > 32) are left out of the sample.
    """
    import threadpoolctl
    from oracle import correlator as OC
    from oracle import geometry as OG
    from oracle import redcal as OR
    done, gerr, t_solve, units = 0, 0.0, 0.0, []
    geo = {}
    for a in arrays:
        if a["n"] <= 32:
            pos = OG.square_positions(a["n"])
            pairs, tix = OG.group_pairs(pos, a["types"])
            geo[a["name"]] = (pos, pairs, tix, OC.canonical_lags(a["n"]))
    # passes over the sampled units until at least min(10 s, budget) of
    # oracle work, stopping within the budget
    min_s = min(10.0, budget_s)
    t0 = time.perf_counter()
    passes, out_of_time = 0, not geo
    while not out_of_time:
        for a in arrays:
            if a["name"] not in geo:
                continue
            pos, pairs, tix, lags = geo[a["name"]]
            types = a["types"]
            for u in a["sample"]:
                volt = a["volt_host"](u)
                if volt.dtype == np.uint8:
                    from synthdata import unpack_ci4
                    re, im = unpack_ci4(volt)
                    v = re.astype(np.float64) + 1j * im.astype(np.float64)
                else:
                    v = volt.astype(np.complex128)
                ts = time.perf_counter()
                vf = OC.fx_correlate(v)
                vred = OC.xengine(vf, pairs)
                cal = OR.calibrate(vred, pos, types, pairs, tix)
                OC.redundant_average(vf, cal["g"], pos, lags)
                t_solve += time.perf_counter() - ts
                done += 1
                # gate: the oracle on the GPU's own V^reduced
                if len(units) < gate_units:
                    ref = OR.calibrate(a["vred_gpu"](u), pos, types, pairs, tix)
                    g = a["gains_gpu"](u)
                    gerr = max(gerr, float(np.max(np.abs(g - ref["g"]) / np.abs(ref["g"]))))
                    units.append(f"{a['name']}:{u}")
                if time.perf_counter() - t0 > budget_s:
                    out_of_time = True
                    break
            if out_of_time:
                break
        passes += 1
        if t_solve >= min_s:
            break
    if done == 0:
        return None, None
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    cpu = {"value": done / t_solve, "unit": "calibrated channel-integrations/s", "cores": threads,
           "kind": "oracle",
           "sample": f"{done} unit solves ({passes} pass(es) over the sampled units of the same workload), "
                     f"one at a time ({t_solve:.1f} s): FX correlator "
                     f"(zgemm), X-engine gather, FIRSTCAL start + dense Gauss-Newton to 1e-10, "
                     f"degeneracy fix, eq. modelvis average"}
    gate = {"max_rel": gerr, "units": units, "tol": 1e-6}
    return cpu, gate


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); units shard across GPUs "
              f"with no collective, so the per-GPU figure is the one to scale.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2005_03060_amd as rrc
    from synthdata import WORKLOADS, workload_voltages
    from synthdata.device import device_voltages

    w = {x.name: x for x in WORKLOADS}[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dtype = "ci4" if w.ci4 else "c64"
    # small workloads: the host generator's exact bytes; large: drawn on the GPU
    host_gen = len(w.grids) == 1 and w.grids[0] * w.grids[0] * w.n_chan * w.n_time <= 64 * 1024 * 1024
    rng = np.random.default_rng(7)
    arrays = []
    for ai, n in enumerate(w.grids):
        if host_gen:
            vnp, g = workload_voltages(w, ai)
            volt = torch.from_numpy(vnp).to(dev)
        else:
            volt, g = device_voltages(w, ai, dev)
        types, npairs = rrc.select_subset(n)
        plan = rrc.Plan(n, types, w.n_chan, w.n_time, dtype=dtype)
        arrays.append(dict(name=f"g{n}", n=n, types=types, npairs=npairs, plan=plan, volt=volt,
                           gains_in=torch.from_numpy(g.astype(np.complex64)).to(dev),
                           out=plan.alloc_outputs(dev),
                           sample=rng.permutation(w.n_chan).tolist()))
    # Batches in flight: consecutive steps alternate over D lanes, each with
    # its own stream, plans (so their own auxiliary streams and workspaces),
    # copy of the input and outputs, so one batch's X-engine and
    # FFT-correlator can run beside the previous batch's latency-bound solve.
    # Lane 0 holds the arrays above; the other lanes copy their inputs.
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    D = args.inflight if args.inflight > 0 else \
        max(1, min(4, -(-cus // (w.n_chan * len(arrays)))))
    lanes = []
    for li in range(D):
        la = arrays if li == 0 else [
            dict(a, plan=rrc.Plan(a["n"], a["types"], w.n_chan, w.n_time, dtype=dtype),
                 volt=a["volt"].clone(), gains_in=a["gains_in"].clone()) for a in arrays]
        for a in la:
            if li:
                a["out"] = a["plan"].alloc_outputs(dev)
            a["plan"].workspace(dev)      # allocated here, not in a timed step
        lanes.append(dict(arrays=la, stream=torch.cuda.Stream(dev),
                          batch=rrc.Batch([a["plan"] for a in la]) if len(la) > 1 else None))
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    batch = lanes[0]["batch"]

    def run_lane(ln):
        if ln["batch"] is None:
            a = ln["arrays"][0]
            a["plan"].run(a["volt"], gains_in=a["gains_in"], mode="pipelined", out=a["out"])
        else:
            la = ln["arrays"]
            ln["batch"].run([a["volt"] for a in la], [a["gains_in"] for a in la],
                            [a["out"] for a in la], mode="pipelined")

    def step(i):
        ln = lanes[i % D]
        with torch.cuda.stream(ln["stream"]):
            run_lane(ln)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for ln in lanes:
        ln["stream"].wait_event(e0)
    for i in range(args.steps):
        step(i)
    for ln in lanes:
        stream.wait_stream(ln["stream"])
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    total_units = w.n_chan * len(arrays)
    value = total_units / (ms * 1e-3)

    # one batch at a time on the launch stream: the time per step when each
    # batch waits for the one before it
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record(stream)
    for _ in range(args.steps):
        run_lane(lanes[0])
    s1.record(stream)
    torch.cuda.synchronize()
    serial_ms = s0.elapsed_time(s1) / args.steps

    # per-stage times with HIP events on the launch stream, each array alone
    def time_fn(fn, reps):
        for _ in range(2):
            fn()
        a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a_.record(stream)
        for _ in range(reps):
            fn()
        b_.record(stream)
        torch.cuda.synchronize()
        return a_.elapsed_time(b_) / reps

    stages = {"xengine": 0.0, "fftcorr": 0.0, "solve": 0.0}
    flops = vbytes = 0.0
    latency = {}
    for a in arrays:
        p = a["plan"]
        stages["xengine"] += time_fn(lambda: p.xengine(a["volt"]), args.steps)
        stages["fftcorr"] += time_fn(lambda: p.fftcorr(a["volt"], a["gains_in"]), args.steps)
        stages["solve"] += time_fn(lambda: p.solve(a["out"]["vred"]), args.steps)
        m = p.info["fft_size"]
        flops += fft_flops_per_sample(a["n"], m) * w.n_time * w.n_chan
        vbytes += (1.0 if w.ci4 else 8.0) * a["n"] ** 2 * w.n_time * w.n_chan
        if len(arrays) > 1:
            # per-array latency of one whole-path run of the array alone
            t = []
            for _ in range(max(5, args.steps)):
                s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s0.record(stream)
                p.run(a["volt"], gains_in=a["gains_in"], mode="pipelined", out=a["out"])
                s1.record(stream)
                torch.cuda.synchronize()
                t.append(s0.elapsed_time(s1))
            latency[a["name"]] = {"p50_ms": float(np.percentile(t, 50)), "p99_ms": float(np.percentile(t, 99))}

    # plain per-channel form: one plan per channel, host sync after each
    plain_ms = None
    if args.plain_steps > 0:
        plain1 = []
        for a in arrays:
            p1 = rrc.Plan(a["n"], a["types"], 1, w.n_time, dtype=dtype)
            plain1.append((a, p1, p1.alloc_outputs(dev)))
        for a, p1, o1 in plain1:
            for c in range(min(2, w.n_chan)):
                p1.run(a["volt"][c:c + 1], gains_in=a["gains_in"][c:c + 1], mode="pipelined", out=o1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            for a, p1, o1 in plain1:
                for c in range(w.n_chan):
                    p1.run(a["volt"][c:c + 1], gains_in=a["gains_in"][c:c + 1], mode="pipelined", out=o1)
                    torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3 / args.plain_steps

    # roofline of the FFT-correlator stage (the O(N log N) core)
    fft_s = stages["fftcorr"] * 1e-3
    roof = {"bound": "alu", "achieved": flops / fft_s / 1e12, "peak": VALU_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": flops / fft_s / 1e12 / VALU_FP32_PEAK_TFLOPS,
            "traffic": measured_traffic(w.name) if len(arrays) == 1 else None,
            "algorithmic_bytes": vbytes,
            "kernel": "k_fftcorr + k_fftfin_fft (FFT-correlator stage)",
            "hbm_achieved_GBs": vbytes / fft_s / 1e9, "hbm_frac": vbytes / fft_s / 1e9 / HBM_PEAK_GBS}
    # the other two stages: the X-engine streams the same voltages (HBM roof);
    # the solve runs one workgroup per unit and is bound by the latency of
    # its serial CG iterations, so its figure is time per unit and CU usage
    x_s = stages["xengine"] * 1e-3
    other = [
        {"kernel": "k_xant + k_xfin (reduced X-engine)", "bound": "hbm",
         "achieved": vbytes / x_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": vbytes / x_s / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes": vbytes},
        {"kernel": "k_solve (reduced redundant calibration)", "bound": "latency",
         "ms_per_launch": stages["solve"], "units_per_launch": total_units,
         "workgroups_per_unit": 1, "cus": cus},
    ]

    status_nonzero = int(sum(int((a["out"]["status"] != 0).sum()) for a in arrays))
    cpu, gate = None, None
    if not args.no_cpu_baseline:
        for a in arrays:
            a["volt_host"] = (lambda u, a=a: a["volt"][u].cpu().numpy())
            a["vred_gpu"] = (lambda u, a=a: (lambda x: x[..., 0] + 1j * x[..., 1] if x.ndim == 2 else x)(
                a["out"]["vred"][u].cpu().numpy()).astype(np.complex128))
            a["gains_gpu"] = (lambda u, a=a: a["out"]["gains"][u].cpu().numpy().astype(np.complex128))
        cpu, gate = cpu_baseline(arrays, args.cpu_seconds, gate_units=4)

    n0 = arrays[0]["n"]
    rec = {
        "metric": METRIC,
        "value": value, "unit": "channel-integrations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "ci4->i32/f32" if w.ci4 else "f32",
        "data": "synthetic" + ("" if host_gen else " (drawn on the GPU)"),
        "config": {"workload": w.name, "grids": [f"{a['n']}x{a['n']}" for a in arrays],
                   "antennas": [a["n"] ** 2 for a in arrays], "channels": w.n_chan, "samples": w.n_time,
                   "fft_size": [a["plan"].info["fft_size"] for a in arrays],
                   "types": [len(a["types"]) for a in arrays], "pairs": [a["npairs"] for a in arrays],
                   "mode": "pipelined, all channels per launch" + (", arrays concurrently" if batch else ""),
                   "batches_in_flight": D,
                   "parallelism": "none (1 GPU)"},
        "stages_ms": stages,
        "one_batch_at_a_time": {"ms_per_step": serial_ms, "value": total_units / (serial_ms * 1e-3)},
        "plain_per_channel": None if plain_ms is None else
        {"ms_per_step": plain_ms, "value": total_units / (plain_ms * 1e-3), "speedup_batched": plain_ms / ms},
        "gain_error_vs_oracle": None if gate is None else dict(gate, status_nonzero=status_nonzero),
        "roofline": roof,
        "roofline_other": other,
        "cpu_baseline": cpu,
    }
    if latency:
        rec["per_array_latency"] = latency
    if n0 and len(arrays) == 1:
        rec["config"].update({"grid": f"{n0}x{n0}", "antennas": n0 * n0})
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
