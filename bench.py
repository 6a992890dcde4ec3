#!/usr/bin/env python3
"""Benchmark: realtime factor and synaptic events/s of the full-scale
microcircuit (77,169 neurons, ~3e8 synapses) on one MI355X.

A bench "step" is one grid step of h = 0.1 ms: drive, update, compaction and
delivery of every spike (one pass of the whole simulation cycle).  Protocol of
the paper's Methods section: the network is instantiated (untimed), 1000 steps
(0.1 s of model time, past the initial transient) are simulated as the
presimulation and discarded, the launch is chosen (autotuner unless
`--launch`), `--warmup` more steps run untimed on it (default 100), then
`--steps` steps are timed (default 100000 = 10 s of model time).
RTF = T_wall / T_model.  Inputs are synthetic (the paper's connectivity table
and initial conditions are not published in it).

Workloads (`--workload`):
  microcircuit  (default) the line above, plus the energy per synaptic event
                (GPU package energy over ~12 s of further simulation), the
                delivery replay, the full-scale adjoint cost per step and the
                CPU oracle baseline;
  balanced      the 5,000-neuron balanced random network, same protocol;
  batched       64 microcircuit instances of scale 0.05-0.25 in one network,
                2 s of model time each, against 64 sequential plain runs;
  adjoint_small / adjoint_full
                adjoint cost per step against the plain forward per step.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import ctypes as C
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H_MS = 0.1
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_persist_microcircuit_hbm_traffic.md")
PERSIST_SRC = os.path.join(ROOT, "paper_2111_04398_amd", "csrc", "mc_persist.hip")


BYTES_PER_EVENT = 9 + 8          # synapse record (target 4, weight 4, delay 1) + one int64 atomic add
BYTES_PER_SPIKE = 16 + 4 + 8     # two row offsets, a spike-list entry, a raster entry
BYTES_PER_NEURON_STEP = 50       # y, I (8 B each) and r (1 B) read and written; ring slot read and cleared


def algorithmic_bytes(events: int, spikes: int, neuron_steps: int) -> int:
    """Bytes the method must move (only what the method itself needs): per
    synaptic event the 9-byte synapse record plus one 8-byte atomic add into
    the ring; per spike its two row offsets, a list entry and a raster
    entry; per neuron-step y, I (8 B) and r (1 B) read and written and its
    ring slot read and cleared."""
    return events * BYTES_PER_EVENT + spikes * BYTES_PER_SPIKE + neuron_steps * BYTES_PER_NEURON_STEP


def measured_traffic(kernel: str, steps_per_launch: int):
    """HBM bytes per step of the persistent kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy), if it
    was taken on the kernel source as it is now; else None."""
    if kernel != "k_persist" or not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    h = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    b = re.search(r"hbm_bytes_per_step:\s*([0-9.eE+]+)", text)
    if not h or not b:
        return None
    if hashlib.sha256(open(PERSIST_SRC, "rb").read()).hexdigest() != h.group(1):
        return None
    per_step = float(b.group(1))
    return {"per_step": per_step, "per_launch": per_step * steps_per_launch}


class DeviceBuffer:
    """Device memory from the HIP runtime that libmc uses (no torch here)."""

    def __init__(self, nbytes: int):
        self.hip = C.CDLL("libamdhip64.so.7")
        self.ptr = C.c_void_p()
        if self.hip.hipMalloc(C.byref(self.ptr), C.c_size_t(nbytes)) != 0:
            raise RuntimeError(f"hipMalloc of {nbytes} bytes failed")

    def free(self):
        if self.ptr:
            self.hip.hipFree(self.ptr)
            self.ptr = C.c_void_p()


class EnergyMeter:
    """Energy of the GPU package the library runs on (compute dies, I/O dies
    and HBM), from the amdsmi energy accumulator.  The accumulator advances
    about once per second with a timestamp of its own, so a sampling thread
    records its updates and a window's power is taken over the whole update
    intervals inside it.  The paper's energy per synaptic event is the energy
    of the simulation phase over its synaptic events; it is reported here both
    whole and above the idle power measured just before (the paper quotes its
    node's power above a baseline).  Unavailable counters leave `error` set."""

    def __init__(self):
        self.h = None
        self.error = None
        self.samples = []            # (host s when first seen, joules, counter ns)
        self._stop = None
        try:
            import amdsmi
            self.smi = amdsmi
            hip = C.CDLL("libamdhip64.so.7")
            buf = C.create_string_buffer(64)
            dev = C.c_int()
            if hip.hipGetDevice(C.byref(dev)) != 0 or hip.hipDeviceGetPCIBusId(buf, 64, dev.value) != 0:
                raise RuntimeError("no HIP device")
            bdf = buf.value.decode().lower()
            amdsmi.amdsmi_init()
            handles = amdsmi.amdsmi_get_processor_handles()
            for h in handles:
                if amdsmi.amdsmi_get_gpu_device_bdf(h).lower() == bdf:
                    self.h = h
            if self.h is None:
                raise RuntimeError(f"device {bdf} not among the {len(handles)} amdsmi processors")
            self._read()
        except Exception as e:   # no counters on this machine: the benchmark runs without them
            self.h = None
            self.error = f"{type(e).__name__}: {e}"

    def _read(self):
        e = self.smi.amdsmi_get_energy_count(self.h)
        return e["energy_accumulator"] * e["counter_resolution"] * 1e-6, e["timestamp"]

    def start(self, period_s: float = 0.005):
        import threading
        self._stop = threading.Event()

        def run():
            while not self._stop.is_set():
                j, ts = self._read()
                self.add(time.perf_counter(), j, ts)
                time.sleep(period_s)

        self._thread = threading.Thread(target=run, daemon=True)
        self._thread.start()

    def add(self, t: float, joules: float, ts: int):
        """Keeps a reading if it is the first or advances the last kept one
        (a rare read returns an unrelated timestamp); repeats are dropped."""
        if self.samples:
            _, j0, ts0 = self.samples[-1]
            if not (ts0 < ts < ts0 + 5_000_000_000 and joules >= j0):
                return
        self.samples.append((t, joules, ts))

    def stop(self):
        if self._stop is not None:
            self._stop.set()
            self._thread.join()
            self._stop = None

    def power(self, t0: float, t1: float, slack: float = 0.01):
        """Mean watts over the accumulator intervals that lie inside host
        times [t0, t1], and the seconds they cover (None if none does)."""
        u = self.samples
        joules = ns = 0
        for a, b in zip(u, u[1:]):
            if a[0] - slack >= t0 and b[0] <= t1:
                joules += b[1] - a[1]
                ns += b[2] - a[2]
        return (joules / (ns * 1e-9), ns * 1e-9) if ns > 0 else (None, 0.0)


def energy_run(net, meter, wall_s_target: float, ms_per_step: float, idle_s: float = 3.2) -> dict:
    """Idle window, then enough steps for about `wall_s_target` seconds; the
    package power of each and the energy per synaptic event of the run."""
    if meter is None or meter.h is None:
        return {"available": False, "error": meter.error if meter else "disabled"}
    steps = max(1000, int(wall_s_target / (ms_per_step * 1e-3)))
    # room for the whole run's raster, so that no drain pauses it (the bound
    # is a worst case: one spike per refractory period per neuron)
    from paper_2111_04398_amd.mc import MCError
    while True:
        try:
            net.reserve(steps)
            break
        except MCError:
            if steps <= 20000:
                raise
            steps //= 2
    meter.start()
    try:
        net.counters()                                  # synchronizes
        i0 = time.perf_counter()
        time.sleep(idle_s)
        i1 = time.perf_counter()
        c0 = net.counters()
        t0 = time.perf_counter()
        net.simulate(steps)
        gpu_ms = net.last_simulate_ms()                 # waits for the steps
        t1 = time.perf_counter()
        c1 = net.counters()
    finally:
        meter.stop()
    p_idle, s_idle = meter.power(i0, i1)
    p_run, s_run = meter.power(t0, t1)
    events = c1["events"] - c0["events"]
    rate = events / (gpu_ms * 1e-3)
    out = {"available": p_run is not None, "source": "amdsmi package energy accumulator (1 Hz updates)",
           "steps": steps, "model_s": steps * H_MS * 1e-3, "wall_s": gpu_ms * 1e-3, "events_per_s": rate,
           "power_w": p_run, "seconds_measured": s_run, "idle_power_w": p_idle, "idle_seconds_measured": s_idle,
           "paper_uj_per_synaptic_event": {"128_threads_1_node": 0.33, "256_threads_2_nodes": 0.48}}
    if p_run is not None:
        out["uj_per_synaptic_event"] = p_run / rate * 1e6
        if p_idle is not None:
            out["uj_per_synaptic_event_above_idle"] = (p_run - p_idle) / rate * 1e6
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mc, workload, launch: dict, presim: int, steps: int, steps_1t: int) -> dict:
    """The CPU oracle as it stands, on this host's cores, over a bounded
    sample of the same workload: `presim` untimed steps, then `steps` timed
    with all threads, then `steps_1t` timed with one thread.  The GPU runs
    the same span from a fresh network (same launch) and its integer event
    and spike counts over the timed span must equal the oracle's."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import oracle  # test infrastructure; only this leg of the benchmark uses it
    if not os.path.exists(os.path.join(ROOT, "oracle", "libmc_oracle.so")):
        oracle.build()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    oracle.set_threads(threads)
    o = oracle.Oracle(workload.to_dict())
    o.run(presim)
    sp0, ev0 = o.counters()
    t = o.run(steps)
    sp1, ev1 = o.counters()
    oracle.set_threads(1)
    t1 = o.run(steps_1t)
    sp2, ev2 = o.counters()
    oracle.set_threads(threads)
    # the same span on the GPU
    g = mc.Network(workload, device_connect=True)
    g.set_launch(**launch)
    g.reserve(presim + steps + steps_1t)
    g.simulate(presim)
    c0 = g.counters()
    g.simulate(steps)
    c1 = g.counters()
    g.simulate(steps_1t)
    c2 = g.counters()
    g.close()
    same = (c1["events"] - c0["events"] == ev1 - ev0 and c2["events"] - c1["events"] == ev2 - ev1 and
            bool(np.array_equal(c1["spikes_per_pop"] - c0["spikes_per_pop"], sp1 - sp0)) and
            bool(np.array_equal(c2["spikes_per_pop"] - c1["spikes_per_pop"], sp2 - sp1)))
    ev, ev_1 = ev1 - ev0, ev2 - ev1
    return {"value": t / (steps * H_MS * 1e-3), "unit": "RTF (host wall s per model s)", "cores": threads,
            "kind": "oracle", "events_per_s": ev / t, "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "one_thread": {"value": t1 / (steps_1t * H_MS * 1e-3), "events_per_s": ev_1 / t1, "steps": steps_1t,
                           "events": ev_1, "seconds": t1},
            "events_equal_gpu": same,
            "sample": f"{workload.name}: {presim} untimed presim steps, then {steps} timed steps "
                      f"({steps * H_MS:g} ms of model time) with {threads} threads ({ev} synaptic events, {t:.2f} s), "
                      f"then {steps_1t} steps with 1 thread ({ev_1} events, {t1:.2f} s)"}


def parse_launch(text: str) -> tuple:
    """scheme,block,neurons_per_wg,steps_per_graph[,rows_per_wave]"""
    v = [int(x) for x in text.split(",")]
    if len(v) not in (4, 5):
        raise SystemExit("--launch takes scheme,block,neurons_per_wg,steps_per_graph[,rows_per_wave]")
    return tuple(v)


def timed_run(net, steps: int, presim: int, warmup: int, launch: str, tune_steps: int):
    """The workload's presimulation (discarded, as in the paper's protocol:
    the measured span starts after 0.1 s of model time, past the initial
    transient), the launch choice, `warmup` untimed steps on that launch,
    then `steps` timed steps.  Returns (gpu ms, events, spikes, host s,
    autotuned)."""
    net.reserve(presim)
    net.simulate(presim)
    if launch:
        net.set_launch(*parse_launch(launch))
        tuned = False
    else:
        net.tune(tune_steps)                  # restores the state it started from
        tuned = True
    if warmup > 0:
        net.reserve(warmup)
        net.simulate(warmup)
    net.reserve(steps)
    c0 = net.counters()                       # synchronizes
    t0 = time.perf_counter()
    net.simulate(steps)
    gpu_ms = net.last_simulate_ms()           # HIP events on the simulation stream (waits for them)
    host_s = time.perf_counter() - t0
    c1 = net.counters()
    return gpu_ms, c1["events"] - c0["events"], c1["spikes"] - c0["spikes"], host_s, tuned


def adjoint_cost(net, window: int, ckpt_every: int, v_target: float, fp32: bool) -> dict:
    """One adjoint window from the network's current state against the plain
    forward of the same window from the same state (same launch): GPU time
    per step of each (the adjoint's forward with checkpoints and its reverse
    pass), with the state restored in between."""
    start = net.save_state()
    net.reserve(window)
    net.counters()
    net.simulate(window)
    plain_ms = net.last_simulate_ms()
    net.load_state(start)
    buf = DeviceBuffer(net.M * (4 if fp32 else 8))
    try:
        t0 = time.perf_counter()
        loss = net.adjoint(window, ckpt_every, v_target, fp32, buf.ptr.value)
        host_s = time.perf_counter() - t0
        fwd, rev = net.last_adjoint_ms()
    finally:
        buf.free()
    return {"window_steps": window, "ckpt_every": ckpt_every, "grad": "f32" if fp32 else "f64", "loss": loss,
            "forward_ms_per_step": fwd / window, "reverse_ms_per_step": rev / window,
            "plain_forward_ms_per_step": plain_ms / window,
            "adjoint_vs_plain": (fwd + rev) / plain_ms,
            "host_s": host_s}


def probes(net, replay_slots: int) -> dict:
    """What the memory system achieves for the delivery's two costs and for
    the persistent kernel's exchange (library microbenchmarks, this run):
    a 4 GiB streaming read; int64 atomic adds into slot-major tables of this
    network's ring stride -- 128 slots (the ring, 79 MB at full scale), the
    replay ring, and ~759 MB (the batched workload's ring) -- uniformly
    random and in the delivery's own row/delay pattern; and the empty
    persistent loop of the scheme in use."""
    out = {"stream_read_gbs": net.probe_stream(4 << 30)}
    stride = (net.N + 63) // 64 * 64
    big = max(128, int(759e6 / 8 / stride))
    atomic = {}
    for slots in sorted({128, replay_slots, big}):
        for pattern, name in ((0, "uniform"), (1, "rows")):
            atomic[f"{slots}x{stride}_{name}"] = net.probe_atomics(slots, pattern) * 1e9
    out["atomic_adds_per_s"] = atomic
    out["atomic_ceiling_per_s"] = max(atomic.values())
    if net.get_launch()["scheme"] == 1:
        out["exchange_us_per_step"] = net.probe_exchange(10000)
    return out


def run_plain(args, mc, w) -> dict:
    t0 = time.perf_counter()
    net = mc.Network(w, device_connect=True)
    build_s = time.perf_counter() - t0
    steps = args.steps or w.sim_steps
    gpu_ms, events, spikes, host_s, tuned = timed_run(net, steps, w.presim_steps, args.warmup, args.launch,
                                                      args.tune_steps)
    kern = net.last_kernel_ms()
    wall_s = gpu_ms * 1e-3
    t_model = steps * H_MS * 1e-3
    launch = net.get_launch()
    persistent = launch["scheme"] == mc.SCHEME_PERSISTENT_LDS and kern["launches"] > 0
    kernel = "k_persist" if persistent else ("k_step" if launch["scheme"] == mc.SCHEME_STEP_KERNELS else "k_step+k_owner")
    alg_bytes_per_step = algorithmic_bytes(events, spikes, net.N * steps) / steps
    # the dominant kernel's own time: the persistent kernel's launches (HIP
    # events around each launch on the simulation stream), else the whole span
    k_ms = kern["ms"] if persistent else gpu_ms
    k_launches = kern["launches"] if persistent else 1
    k_us_per_step = k_ms * 1e3 / steps
    avg_launch_ms = k_ms / k_launches
    steps_per_launch = steps / k_launches
    achieved_gbs = alg_bytes_per_step * steps_per_launch / (avg_launch_ms * 1e-3) / 1e9
    full = w.name == "microcircuit"
    tr = measured_traffic(kernel, int(round(steps_per_launch))) if full else None   # counters were taken on this workload
    # replay span: 1000 recorded steps after the presim, simulated (untimed) if the timed span was shorter
    rs = args.replay_steps
    r0 = w.presim_steps
    need = r0 + rs - net.counters()["step"]
    if need > 0:
        net.reserve(need)
        net.simulate(need)
    pr = probes(net, rs + 101) if not args.no_probes else {}
    hbm = {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved_gbs / HBM_PEAK_GBS,
           "alg_bytes_per_step": alg_bytes_per_step,
           "bytes_per_unit": {"event": BYTES_PER_EVENT, "spike": BYTES_PER_SPIKE, "neuron_step": BYTES_PER_NEURON_STEP},
           "traffic": tr["per_launch"] if tr else None,
           "traffic_per_step": tr["per_step"] if tr else None,
           "traffic_source": os.path.relpath(TRAFFIC_FILE, ROOT) if tr else None}
    if pr:
        hbm["measured_stream_read_gbs"] = pr["stream_read_gbs"]
        hbm["frac_of_measured_read"] = achieved_gbs / pr["stream_read_gbs"]
    if persistent and pr.get("exchange_us_per_step"):
        floor = pr["exchange_us_per_step"]
        roofline = {"bound": "latency", "kernel": kernel, "achieved": 1e6 / k_us_per_step,
                    "peak": 1e6 / floor, "unit": "steps/s", "frac": floor / k_us_per_step,
                    "traffic": hbm["traffic"], "kernel_us_per_step": k_us_per_step,
                    "floor_us_per_step": floor,
                    "floor": "empty persistent loop of the same workgroups exchanging one record per step",
                    "launches": k_launches, "steps_per_launch": steps_per_launch, "avg_launch_ms": avg_launch_ms,
                    "hbm": hbm}
    else:
        roofline = {"bound": "hbm", "kernel": kernel, **hbm, "kernel_us_per_step": k_us_per_step,
                    "launches": k_launches, "steps_per_launch": steps_per_launch, "avg_launch_ms": avg_launch_ms}
    out = {
        "metric": "realtime factor + synaptic events/s, full microcircuit 77k neurons/3e8 syn" if full else
                  f"realtime factor + synaptic events/s, {w.name} ({net.N} neurons, {net.M} synapses)",
        # the paper's headline figure (Table 1): wall time per model time.  The
        # events/s of a short window follow the network's population rhythm
        # (bursts every ~46 ms), the time per step hardly does
        "value": wall_s / t_model,
        "unit": "RTF (GPU wall s per model s)",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": gpu_ms / steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+i64",
        "data": "synthetic",
        "config": {"workload": w.name, "neurons": net.N, "synapses": net.M, "h_ms": H_MS,
                   "t_model_s": t_model, "presim_steps": w.presim_steps, "launch": launch, "autotuned": tuned,
                   "persist_shape": net.persist_shape()},
        "rtf": wall_s / t_model,
        "rtf_host_clock": host_s / t_model,
        "events": events,
        "spikes": spikes,
        "events_per_s": events / wall_s,
        "mean_rate_hz": spikes / net.N / t_model,
        "build_s": build_s,
        "roofline": roofline,
        "paper_context": {"rtf_2x64_core_epyc_node": 0.67, "rtf_2_nodes": 0.53},
    }
    if pr:
        out["probes"] = pr
    if args.energy_wall > 0:
        out["energy"] = energy_run(net, EnergyMeter(), args.energy_wall, gpu_ms / steps)
    # throughput form of the delivery: the recorded spikes of rs steps in one launch
    if rs > 0:
        r_ms, r_ev, _ = net.replay_delivery(r0, r0 + rs)
        r_rate = r_ev / (r_ms * 1e-3)
        r_gbs = r_ev * BYTES_PER_EVENT / (r_ms * 1e-3) / 1e9
        rep = {"kernel": "k_replay", "steps": rs, "events": r_ev, "ms": r_ms, "events_per_s": r_rate,
               "achieved_gbs": r_gbs, "frac_hbm": r_gbs / HBM_PEAK_GBS}
        if pr:
            key = f"{rs + 101}x{(net.N + 63) // 64 * 64}_rows"
            rep["atomic_ceiling_per_s"] = pr["atomic_ceiling_per_s"]
            rep["frac_atomic"] = r_rate / pr["atomic_ceiling_per_s"]
            rep["same_table_rows_probe_per_s"] = pr["atomic_adds_per_s"].get(key)
            rep["frac_hbm_measured"] = r_gbs / pr["stream_read_gbs"]
        out["delivery_replay"] = rep
    if args.phases and launch["scheme"] in (mc.SCHEME_PERSISTENT_LDS, mc.SCHEME_PERSISTENT_BUCKETS):
        out["phases_us_per_step"] = net.profile_phases(args.phases)
    if args.adjoint_window > 0 and full:
        out["adjoint"] = adjoint_cost(net, args.adjoint_window, 100, -58.0, True)
    net.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mc, w, launch, presim=1000, steps=args.cpu_steps, steps_1t=args.cpu_steps_1t)
    return out


def run_batched(args, mc, w) -> dict:
    """All instances in one network (one launch per graph of steps) against
    the same instances simulated one after another as plain networks."""
    steps = args.steps or w.sim_steps
    t0 = time.perf_counter()
    net = mc.Network(w, device_connect=True)
    build_s = time.perf_counter() - t0
    gpu_ms, events, spikes, host_s, tuned = timed_run(net, steps, w.presim_steps, args.warmup, args.launch,
                                                      args.tune_steps)
    launch = net.get_launch()
    N, M, n_inst = net.N, net.M, net.n_instances
    energy = energy_run(net, EnergyMeter(), args.energy_wall, gpu_ms / steps) if args.energy_wall > 0 else None
    phases = None
    if args.phases and launch["scheme"] in (mc.SCHEME_PERSISTENT_LDS, mc.SCHEME_PERSISTENT_BUCKETS):
        phases = net.profile_phases(args.phases)
    net.close()
    seq_ms, seq_events, seq_launch = 0.0, 0, {}
    n_seq = n_inst if args.seq_instances <= 0 else min(args.seq_instances, n_inst)
    for b in range(n_seq):
        one = mc.Network(w.instance(b), device_connect=True)
        ms, ev, _, _, _ = timed_run(one, steps, w.presim_steps, args.warmup, args.seq_launch, args.tune_steps)
        seq_ms += ms
        seq_events += ev
        lc = one.get_launch()
        key = f"{lc['scheme']},{lc['block']},{lc['neurons_per_wg']},{lc['steps_per_graph']}"
        seq_launch[key] = seq_launch.get(key, 0) + 1
        one.close()
    seq_ms_all = seq_ms * n_inst / n_seq
    wall_s = gpu_ms * 1e-3
    return {
        "metric": "instances/s, 64 batched microcircuit instances (scale 0.05-0.25), 2 s model time each",
        "value": n_inst / wall_s,
        "unit": "instances/s",
        "n_gpus": 1, "steps": steps, "warmup": args.warmup, "ms_per_step": gpu_ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+i64", "data": "synthetic",
        "config": {"workload": w.name, "instances": n_inst, "neurons": N, "synapses": M, "h_ms": H_MS,
                   "t_model_s_each": steps * H_MS * 1e-3, "presim_steps": w.presim_steps, "launch": launch,
                   "autotuned": tuned},
        "events": events, "spikes": spikes, "events_per_s": events / wall_s,
        "build_s": build_s,
        "sequential": {"instances_timed": n_seq, "gpu_s": seq_ms * 1e-3, "gpu_s_all": seq_ms_all * 1e-3,
                       "instances_per_s": n_inst / (seq_ms_all * 1e-3), "events": seq_events,
                       "launches": seq_launch},
        "speedup_vs_sequential": (seq_ms_all * 1e-3) / wall_s,
        "energy": energy,
        "phases_us_per_step": phases,
    }


def run_adjoint(args, mc, w) -> dict:
    """Adjoint over the workload's window from a fresh network against the
    plain forward of the same window from the same state (same launch)."""
    S, K = w.adj_window, w.adj_ckpt_every
    net = mc.Network(w, device_connect=True)
    if args.launch:
        net.set_launch(*parse_launch(args.launch))
    else:
        net.tune(min(args.tune_steps, S))
    launch = net.get_launch()
    a = adjoint_cost(net, S, K, w.adj_v_target, w.adj_fp32)
    c = net.counters()
    net.close()
    return {
        "metric": "adjoint ms per step vs plain forward ms per step",
        "value": a["forward_ms_per_step"] + a["reverse_ms_per_step"],
        "unit": "ms/step",
        "n_gpus": 1, "steps": S, "warmup": 0, "ms_per_step": a["forward_ms_per_step"] + a["reverse_ms_per_step"],
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" + ("->f32 grad" if w.adj_fp32 else ""), "data": "synthetic",
        "config": {"workload": w.name, "window_steps": S, "ckpt_every": K, "launch": launch},
        "adjoint": a, "spikes": int(sum(c["spikes_per_pop"])), "events": c["events"],
    }


def run_build_compare(args, mc, w) -> dict:
    """Instantiation of the workload with the connections drawn on the host
    and on the device (MC_FLAG_DEVICE_CONNECT), timed by the host clock, and
    the two synapse stores compared bit for bit."""
    import numpy as np
    t0 = time.perf_counter()
    a = mc.Network(w)
    host_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = mc.Network(w, device_connect=True)
    dev_s = time.perf_counter() - t0
    same = all(np.array_equal(x, y) for x, y in zip(a.synapses(), b.synapses()))
    n, m = a.N, a.M
    a.close()
    b.close()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"metric": f"network instantiation seconds, {w.name} ({n} neurons, {m} synapses)", "value": dev_s,
            "unit": "s", "n_gpus": 1, "steps": 0, "warmup": 0, "ms_per_step": None, "higher_is_better": False,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64 (Philox pair tests)", "data": "synthetic",
            "config": {"workload": w.name, "neurons": n, "synapses": m},
            "host_draws_s": host_s, "device_draws_s": dev_s, "speedup": host_s / dev_s, "host_threads": threads,
            "identical_store": same}


def copy_calibration(nbytes: int) -> None:
    """A plain device-to-device copy of known size (the HIP runtime's copy
    kernel, called through the runtime libmc already loaded): reads nbytes
    and writes nbytes per copy.  Its HBM byte counters give the scale of the
    counters taken on the simulation kernels."""
    src, dst = DeviceBuffer(nbytes), DeviceBuffer(nbytes)
    hip = src.hip
    ok = hip.hipMemset(src.ptr, 1, C.c_size_t(nbytes)) == 0 and hip.hipDeviceSynchronize() == 0
    for _ in range(3):
        ok = ok and hip.hipMemcpy(dst.ptr, src.ptr, C.c_size_t(nbytes), 3) == 0   # hipMemcpyDeviceToDevice
    ok = ok and hip.hipDeviceSynchronize() == 0
    src.free()
    dst.free()
    if not ok:
        raise RuntimeError("copy calibration failed")
    print(json.dumps({"copy_calibration_bytes": nbytes, "copies": 3}), flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0,
                    help="timed steps (default: the workload's span, 100000 = 10 s for the microcircuit)")
    ap.add_argument("--warmup", type=int, default=100,
                    help="untimed steps on the chosen launch after the workload's presimulation (1000 steps)")
    ap.add_argument("--workload", default="microcircuit",
                    choices=["microcircuit", "balanced", "batched", "adjoint_small", "adjoint_full"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--energy-wall", type=float, default=12.0, metavar="S",
                    help="after timing: idle power, then about S seconds of simulation under the package "
                         "energy counter for the energy per synaptic event (0: skip)")
    ap.add_argument("--cpu-steps", type=int, default=15000, help="oracle steps timed with all host threads")
    ap.add_argument("--cpu-steps-1t", type=int, default=600, help="oracle steps timed with one thread")
    ap.add_argument("--no-probes", action="store_true", help="skip the stream/atomic/exchange microbenchmarks")
    ap.add_argument("--launch", default="",
                    help="scheme,block,neurons_per_wg,steps_per_graph[,rows_per_wave] (default: autotuned)")
    ap.add_argument("--tune-steps", type=int, default=2000, help="steps per autotuner candidate")
    ap.add_argument("--replay-steps", type=int, default=1000, help="steps of raster replayed in one launch")
    ap.add_argument("--phases", type=int, default=0, help="after timing, profile this many steps per phase")
    ap.add_argument("--adjoint-window", type=int, default=2000,
                    help="microcircuit: steps of the full-scale FP32 adjoint timed after the run (0: skip)")
    ap.add_argument("--seq-instances", type=int, default=0,
                    help="batched: instances timed sequentially (0: all; the total is scaled to all)")
    ap.add_argument("--seq-launch", default="", help="batched: launch of the sequential runs (default: autotuned)")
    ap.add_argument("--compare-build", action="store_true",
                    help="only time the workload's instantiation with host and with device connection draws")
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
    w = workloads.PRESETS[args.workload]()
    if args.compare_build:
        out = run_build_compare(args, mc, w)
    elif args.workload in ("microcircuit", "balanced"):
        out = run_plain(args, mc, w)
    elif args.workload == "batched":
        out = run_batched(args, mc, w)
    else:
        out = run_adjoint(args, mc, w)
    print(json.dumps(out), flush=True)
    if args.copy_calibration > 0:
        copy_calibration(args.copy_calibration << 20)
    return 0


if __name__ == "__main__":
    sys.exit(main())
