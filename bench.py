"""Throughput of the calibrated FFT-correlator on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

One step = one integration of every unit (array, channel) of the workload
through the whole hot path: reduced X-engine, FFT-correlator (gain
application, padded spatial FFT, |.|^2 integration, inverse transform and
redundant normalisation) and the reduced redundant calibration solve.  The
batched path issues the steps for all units at once (rrc_run, PIPELINED: the
FFT applies the previous integration's gains); the plain path calibrates one
channel at a time, synchronising after each.  Inputs are resident in HBM
before timing starts.  Prints one JSON line.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="g16_c64_t1024")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--plain-steps", type=int, default=2)
    return ap.parse_args()


def cpu_baseline(w, volt_np, types, budget_s):
    """The FP64 oracle, as it stands, on a bounded sample of the same units."""
    import threadpoolctl
    from oracle import correlator as OC
    from oracle import geometry as OG
    from oracle import redcal as OR
    n = w.grids[0]
    pos = OG.square_positions(n)
    pairs, tix = OG.group_pairs(pos, types)
    lags = OC.canonical_lags(n)
    done, t0 = 0, time.perf_counter()
    while done < volt_np.shape[0]:
        v = volt_np[done].astype(np.complex128)
        vf = OC.fx_correlate(v)
        vred = OC.xengine(vf, pairs)
        cal = OR.calibrate(vred, pos, types, pairs, tix)
        OC.redundant_average(vf, cal["g"], pos, lags)
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    info = threadpoolctl.threadpool_info()
    threads = max([i.get("num_threads", 1) for i in info] + [1])
    return {"value": done / dt, "unit": "calibrated channel-integrations/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{done} of {volt_np.shape[0]} units of the same workload, one at a time "
                      f"({dt:.1f} s): FX correlator (zgemm), X-engine gather, FIRSTCAL start + dense "
                      f"Gauss-Newton to 1e-10, degeneracy fix, eq. modelvis average"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); units shard across GPUs "
              f"with no collective, so the per-GPU figure is the one to scale.", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2005_03060_amd as rrc
    from synthdata import WORKLOADS, workload_voltages

    w = {x.name: x for x in WORKLOADS}[args.workload]
    if len(w.grids) != 1 or w.ci4:
        raise SystemExit(f"workload {w.name} is not supported by bench.py yet")
    n = w.grids[0]
    U, T = w.n_chan, w.n_time
    t_gen = time.perf_counter()
    volt_np, gains_np = workload_voltages(w, 0)
    t_gen = time.perf_counter() - t_gen
    types, npairs = rrc.select_subset(n)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    volt = torch.from_numpy(volt_np).to(dev)
    gains_in = torch.from_numpy(gains_np.astype(np.complex64)).to(dev)
    plan = rrc.Plan(n, types, U, T)
    out = plan.alloc_outputs(dev)
    stream = torch.cuda.current_stream()

    def step():
        plan.run(volt, gains_in=gains_in, mode="pipelined", out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    value = U / (ms * 1e-3)

    # per-stage times with HIP events on the launch stream
    def time_stage(fn, reps):
        for _ in range(2):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    vred = out["vred"]
    ws = plan.workspace(dev)
    stage_ms = {
        "xengine": time_stage(lambda: plan.xengine(volt), args.steps),
        "fftcorr": time_stage(lambda: plan.fftcorr(volt, gains_in), args.steps),
        "solve": time_stage(lambda: plan.solve(vred), args.steps),
    }
    del ws

    # plain per-channel form: one plan per channel, host sync after each
    plan1 = rrc.Plan(n, types, 1, T)
    out1 = plan1.alloc_outputs(dev)
    plain_ms = None
    if args.plain_steps > 0:
        for c in range(2):
            plan1.run(volt[c:c + 1], gains_in=gains_in[c:c + 1], mode="pipelined", out=out1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.plain_steps):
            for c in range(U):
                plan1.run(volt[c:c + 1], gains_in=gains_in[c:c + 1], mode="pipelined", out=out1)
                torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3 / args.plain_steps

    # accuracy gate on a seeded sample of units: gains vs the oracle
    from oracle import geometry as OG
    from oracle import redcal as OR
    pos = OG.square_positions(n)
    pairs, tix = OG.group_pairs(pos, types)
    rng = np.random.default_rng(7)
    sample = sorted(rng.choice(U, size=min(U, 4), replace=False).tolist())
    gerr = 0.0
    st = out["status"].cpu().numpy()
    for u in sample:
        ref = OR.calibrate(out["vred"][u].cpu().numpy().astype(np.complex128), pos, types, pairs, tix)
        g = out["gains"][u].cpu().numpy().astype(np.complex128)
        gerr = max(gerr, float(np.max(np.abs(g - ref["g"]) / np.abs(ref["g"]))))

    # roofline of the FFT-correlator stage (the O(N log N) core)
    m = plan.info["fft_size"]
    flops = fft_flops_per_sample(n, m) * T * U
    vbytes = 8.0 * n * n * T * U
    fft_s = stage_ms["fftcorr"] * 1e-3
    roof = {"bound": "alu", "achieved": flops / fft_s / 1e12, "peak": VALU_FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": flops / fft_s / 1e12 / VALU_FP32_PEAK_TFLOPS, "traffic": None,
            "kernel": "k_fftcorr + k_fftfin (fftcorr stage)",
            "hbm_achieved_GBs": vbytes / fft_s / 1e9, "hbm_frac": vbytes / fft_s / 1e9 / HBM_PEAK_GBS}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, volt_np, types, args.cpu_seconds)

    rec = {
        "metric": "calibrated channel-integrations/sec (batched+adjoint vs plain) at stated gain error",
        "value": value, "unit": "channel-integrations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{n}x{n}", "antennas": n * n, "channels": U,
                   "samples": T, "fft_size": m, "types": len(types), "pairs": npairs,
                   "mode": "pipelined, all channels per launch", "parallelism": "none (1 GPU)"},
        "stages_ms": stage_ms,
        "plain_per_channel": None if plain_ms is None else
        {"ms_per_step": plain_ms, "value": U / (plain_ms * 1e-3), "speedup_batched": plain_ms / ms},
        "gain_error_vs_oracle": {"max_rel": gerr, "units": sample, "tol": 1e-6,
                                 "status_nonzero": int(np.sum(st != 0))},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
