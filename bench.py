#!/usr/bin/env python3
"""Benchmark: realtime factor and synaptic events/s of the full-scale
microcircuit (77,169 neurons, ~3e8 synapses) on one MI355X.

A bench "step" is one grid step of h = 0.1 ms: drive, update, compaction and
delivery of every spike (one pass of the whole simulation cycle).  Protocol of
the paper's Methods section: the network is instantiated (untimed), `--warmup`
steps are simulated as the presimulation (default 1000 = 0.1 s, discarded),
then `--steps` steps are timed (default 100000 = 10 s of model time).
RTF = T_wall / T_model.  Inputs are synthetic (the paper's connectivity table
and initial conditions are not published in it): see the design doc.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H_MS = 0.1
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(events: int, spikes: int, neuron_steps: int) -> int:
    """Bytes the method must move: per synaptic event the 9-byte synapse
    record (target 4, weight 4, delay 1) plus an 8-byte read-modify-write of
    the ring entry (16 B); per spike its two row offsets (16 B), a list entry
    (4 B) and a raster entry (8 B); per neuron-step y, I, r read and written
    (2 x 20 B) and its ring slot read and cleared (2 x 8 B)."""
    return events * (9 + 16) + spikes * (16 + 4 + 8) + neuron_steps * (40 + 16)


def cpu_baseline(workload, presim: int, steps: int) -> dict:
    """The CPU oracle as it stands, on this host's cores, over a bounded
    sample of the same workload: `presim` untimed steps, then `steps` timed."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle  # test infrastructure; only this leg of the benchmark uses it
    if not os.path.exists(os.path.join(ROOT, "oracle", "libmc_oracle.so")):
        oracle.build()
    o = oracle.Oracle(workload.to_dict())
    o.run(presim)
    ev0 = o.counters()[1]
    t = o.run(steps)
    ev = o.counters()[1] - ev0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": ev / t, "unit": "synaptic events/s", "cores": threads, "kind": "oracle",
            "rtf": t / (steps * H_MS * 1e-3),
            "sample": f"{workload.name}: {presim} untimed presim steps, then {steps} timed steps "
                      f"({steps * H_MS:g} ms of model time), {ev} synaptic events, {t:.2f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100000)
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="microcircuit", choices=["microcircuit", "balanced"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=15000)
    ap.add_argument("--launch", default="", help="scheme,block,neurons_per_wg,steps_per_graph (default: autotuned)")
    ap.add_argument("--tune-steps", type=int, default=2000, help="steps per autotuner candidate")
    ap.add_argument("--replay-steps", type=int, default=1000, help="steps of raster replayed in one launch")
    ap.add_argument("--phases", type=int, default=0, help="after timing, profile this many steps per phase")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="at the end, copy a MIB-MiB device buffer 3 times (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design in DESIGN.md, not an executable path", file=sys.stderr)
        return 2

    from paper_2111_04398_amd import mc, workloads
    if not os.path.exists(mc.LIB_PATH):
        from paper_2111_04398_amd import build as _b
        _b.build()
    w = workloads.microcircuit() if args.workload == "microcircuit" else workloads.balanced()

    t0 = time.perf_counter()
    net = mc.Network(w)
    build_s = time.perf_counter() - t0
    net.simulate(args.warmup)                 # presimulation, discarded from timing
    if args.launch:
        s, b, npw, spg = (int(v) for v in args.launch.split(","))
        net.set_launch(scheme=s, block=b, neurons_per_wg=npw, steps_per_graph=spg)
        tuned = False
    else:
        net.tune(args.tune_steps)             # restores the state it started from
        tuned = True
    net.reserve(args.steps)
    c0 = net.counters()                       # synchronizes
    t0 = time.perf_counter()
    net.simulate(args.steps)
    gpu_ms = net.last_simulate_ms()           # HIP events on the simulation stream
    t1 = time.perf_counter()
    c1 = net.counters()
    events = c1["events"] - c0["events"]
    spikes = c1["spikes"] - c0["spikes"]
    wall_s = gpu_ms * 1e-3
    t_model = args.steps * H_MS * 1e-3
    launch = net.get_launch()

    per_step_s = wall_s / args.steps
    alg_bytes_per_step = algorithmic_bytes(events, spikes, net.N * args.steps) / args.steps
    achieved_gbs = alg_bytes_per_step / per_step_s / 1e9
    kernel = "k_step" if launch["scheme"] == mc.SCHEME_STEP_KERNELS else "k_persist"
    out = {
        "metric": "realtime factor + synaptic events/s, full microcircuit 77k neurons/3e8 syn",
        "value": events / wall_s,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+i64",
        "data": "synthetic",
        "config": {"workload": w.name, "neurons": net.N, "synapses": net.M, "h_ms": H_MS,
                   "t_model_s": t_model, "presim_steps": args.warmup, "launch": launch, "autotuned": tuned},
        "rtf": wall_s / t_model,
        "rtf_host_clock": (t1 - t0) / t_model,
        "events": events,
        "spikes": spikes,
        "mean_rate_hz": spikes / net.N / t_model,
        "build_s": build_s,
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved_gbs,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved_gbs / HBM_PEAK_GBS,
            "traffic": None,
            "alg_bytes_per_step": alg_bytes_per_step,
            "atomics_per_s": events / wall_s,
        },
        "paper_context": {"rtf_2x64_core_epyc_node": 0.67, "rtf_2_nodes": 0.53},
    }
    # throughput form of the delivery: recorded spikes of replay-steps steps in one launch
    rs = min(args.replay_steps, args.steps)
    if rs > 0:
        r_ms, r_ev, _ = net.replay_delivery(args.warmup, args.warmup + rs)
        peak = net.atomic_rate(net.N * (rs + 101))
        r_rate = r_ev / (r_ms * 1e-3)
        r_gbs = r_ev * (9 + 16) / (r_ms * 1e-3) / 1e9
        out["delivery_replay"] = {
            "kernel": "k_replay", "steps": rs, "events": r_ev, "ms": r_ms,
            "events_per_s": r_rate, "atomic_peak_per_s": peak * 1e9, "frac_atomic": r_rate / (peak * 1e9),
            "achieved_gbs": r_gbs, "frac_hbm": r_gbs / HBM_PEAK_GBS,
        }
    if args.phases and launch["scheme"] == mc.SCHEME_PERSISTENT_LDS:
        out["phases_us_per_step"] = net.profile_phases(args.phases)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, presim=1000, steps=args.cpu_steps)
    print(json.dumps(out), flush=True)
    net.close()
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration << 20)
    return 0


def copy_calibration(nbytes: int) -> None:
    """A plain device-to-device copy of known size (the HIP runtime's copy
    kernel, called through the runtime libmc already loaded): reads nbytes
    and writes nbytes per copy.  Its HBM byte counters give the scale of the
    counters taken on the simulation kernels."""
    import ctypes as C
    hip = C.CDLL("libamdhip64.so.7")
    src, dst = C.c_void_p(), C.c_void_p()
    for p in (src, dst):
        if hip.hipMalloc(C.byref(p), C.c_size_t(nbytes)) != 0:
            raise RuntimeError("hipMalloc failed")
    ok = hip.hipMemset(src, 1, C.c_size_t(nbytes)) == 0 and hip.hipDeviceSynchronize() == 0
    for _ in range(3):
        ok = ok and hip.hipMemcpy(dst, src, C.c_size_t(nbytes), 3) == 0   # hipMemcpyDeviceToDevice
    ok = ok and hip.hipDeviceSynchronize() == 0
    hip.hipFree(src)
    hip.hipFree(dst)
    if not ok:
        raise RuntimeError("copy calibration failed")
    print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)


if __name__ == "__main__":
    sys.exit(main())
