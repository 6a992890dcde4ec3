"""Python binding of libmc (include/mc.h): argument marshalling only.

Every step of the simulation runs in the HIP kernels of ``libmc.so``; this
module converts numpy arrays and ``Workload`` presets to the C structures and
raises ``MCError`` on any non-zero status.  It never falls back to another
implementation: if the shared library is missing it raises at import of the
first call.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from typing import Optional

import numpy as np

from .workloads import Workload

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmc.so")

MC_OK = 0
MC_ERR_INVALID_ARG = -1
MC_ERR_BUFFER_TOO_SMALL = -6
MC_ERR_MISMATCH = -8
MC_ERR_RANGE = -2
MC_ERR_STATE = -5
MC_ERR_TIMEOUT = -9
MC_MAX_POPS = 16
RING_SLOTS = 128
RULE_FIXED_INDEGREE, RULE_BERNOULLI = 0, 1
GRAD_F64, GRAD_F32 = 0, 1
ADJ_INPUT_AUTO, ADJ_INPUT_RECORD, ADJ_INPUT_REPLAY = 0, 1, 2
FLAG_HOST_ONLY = 1
FLAG_DEVICE_CONNECT = 2
SCHEME_STEP_KERNELS, SCHEME_PERSISTENT_LDS, SCHEME_TARGET_OWNER, SCHEME_PERSISTENT_BUCKETS = 0, 1, 2, 3

ERROR_NAMES = {0: "MC_OK", -1: "MC_ERR_INVALID_ARG", -2: "MC_ERR_RANGE", -3: "MC_ERR_OOM", -4: "MC_ERR_HIP",
               -5: "MC_ERR_STATE", -6: "MC_ERR_BUFFER_TOO_SMALL", -7: "MC_ERR_NO_DEVICE", -8: "MC_ERR_MISMATCH",
               -9: "MC_ERR_TIMEOUT"}


class MCError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class mc_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("n_pops", C.c_int32), ("pop_size", C.POINTER(C.c_int32)),
        ("rule", C.c_int32), ("conn", C.POINTER(C.c_double)), ("w_mean_pA", C.POINTER(C.c_double)),
        ("w_rel_sd", C.c_double), ("d_mean_ms", C.POINTER(C.c_double)), ("d_rel_sd", C.c_double),
        ("d_min_steps", C.c_int32), ("d_max_steps", C.c_int32), ("k_ext", C.POINTER(C.c_double)),
        ("nu_ext_hz", C.c_double), ("w_ext_pA", C.c_double),
        ("tau_m_ms", C.c_double), ("c_m_pF", C.c_double), ("e_l_mV", C.c_double), ("v_reset_mV", C.c_double),
        ("v_th_mV", C.c_double), ("t_ref_ms", C.c_double), ("tau_syn_ms", C.c_double), ("i_e_pA", C.c_double),
        ("h_ms", C.c_double), ("v0_lo_mV", C.c_double), ("v0_hi_mV", C.c_double),
        ("n_instances", C.c_int32), ("inst_scale", C.POINTER(C.c_double)), ("inst_seed", C.POINTER(C.c_uint64)),
        ("hip_stream", C.c_void_p), ("flags", C.c_uint32),
        ("dev_alloc", C.c_void_p), ("dev_free", C.c_void_p), ("alloc_ctx", C.c_void_p),
    ]


#: allocator hook types of mc_config
DEV_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class mc_launch(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("scheme", C.c_int32), ("block", C.c_int32),
                ("neurons_per_wg", C.c_int32), ("steps_per_graph", C.c_int32), ("rows_per_wave", C.c_int32)]


class mc_counters(C.Structure):
    _fields_ = [("step", C.c_int64), ("spikes", C.c_int64), ("events", C.c_int64),
                ("spikes_per_pop", C.c_int64 * MC_MAX_POPS)]


class mc_adjoint_config(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("window_steps", C.c_int64), ("ckpt_every", C.c_int64),
                ("v_target_mV", C.c_double), ("grad_dtype", C.c_int32), ("input_mode", C.c_int32)]


#: every symbol include/mc.h declares
EXPORTS = [
    "mc_build_network", "mc_simulate", "mc_get_spikes", "mc_adjoint", "mc_free", "mc_strerror", "mc_last_error",
    "mc_abi_version", "mc_get_sizes", "mc_get_instance_offsets", "mc_get_pop_offsets", "mc_get_synapses",
    "mc_get_state", "mc_set_state", "mc_get_ring", "mc_inject", "mc_get_propagators", "mc_get_drive_tables",
    "mc_get_counters", "mc_set_launch", "mc_get_launch", "mc_tune", "mc_last_simulate_ms", "mc_reserve",
    "mc_save_state", "mc_load_state", "mc_set_weights", "mc_stream", "mc_profile_phases", "mc_replay_delivery",
    "mc_atomic_rate", "mc_last_adjoint_ms", "mc_get_persist_shape", "mc_get_phase_table", "mc_apply_gradient",
    "mc_last_kernel_ms", "mc_probe_stream", "mc_probe_atomics", "mc_probe_exchange", "mc_simulate_noalloc",
]

_lib = None
loaded_after_torch = False


def lib() -> C.CDLL:
    """Loads libmc.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2111_04398_amd/build.py (or __graft_entry__.build())")
    # libmc links the HIP runtime by soname.  If torch (which ships its own
    # runtime under another file name) is already imported, that runtime
    # serves libmc too; torch imported *after* this point would bring a
    # second runtime into the process, which the torch binding refuses.
    global loaded_after_torch
    loaded_after_torch = "torch" in sys.modules
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = np.ctypeslib.ndpointer
    L.mc_build_network.argtypes = [C.POINTER(mc_config), C.POINTER(vp)]
    L.mc_simulate.argtypes = [vp, i64]
    L.mc_simulate_noalloc.argtypes = [vp, i64]
    L.mc_get_spikes.argtypes = [vp, i64, i64, vp, vp, i64, C.POINTER(i64)]
    L.mc_adjoint.argtypes = [vp, C.POINTER(mc_adjoint_config), vp, C.POINTER(f64)]
    L.mc_free.argtypes = [vp]
    L.mc_free.restype = None
    L.mc_strerror.argtypes = [C.c_int]
    L.mc_strerror.restype = C.c_char_p
    L.mc_last_error.argtypes = []
    L.mc_last_error.restype = C.c_char_p
    L.mc_abi_version.restype = C.c_int
    L.mc_get_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]
    L.mc_get_instance_offsets.argtypes = [vp, P(np.int64)]
    L.mc_get_pop_offsets.argtypes = [vp, i32, P(np.int64)]
    L.mc_get_synapses.argtypes = [vp, vp, vp, vp, vp]
    L.mc_get_state.argtypes = [vp, vp, vp, vp]
    L.mc_set_state.argtypes = [vp, P(np.float64), P(np.float64), P(np.int32)]
    L.mc_get_ring.argtypes = [vp, i64, P(np.int64)]
    L.mc_inject.argtypes = [vp, i64, i64, i64]
    L.mc_get_propagators.argtypes = [vp, P(np.float64)]
    L.mc_get_drive_tables.argtypes = [vp, P(np.uint64)]
    L.mc_get_counters.argtypes = [vp, C.POINTER(mc_counters)]
    L.mc_set_launch.argtypes = [vp, C.POINTER(mc_launch)]
    L.mc_get_launch.argtypes = [vp, C.POINTER(mc_launch)]
    L.mc_tune.argtypes = [vp, i64, C.POINTER(mc_launch)]
    L.mc_last_simulate_ms.argtypes = [vp, C.POINTER(f64)]
    L.mc_last_kernel_ms.argtypes = [vp, C.POINTER(f64), C.POINTER(i64), C.POINTER(i64)]
    L.mc_probe_stream.argtypes = [vp, i64, C.POINTER(f64)]
    L.mc_probe_atomics.argtypes = [vp, i64, i32, C.POINTER(f64)]
    L.mc_probe_exchange.argtypes = [vp, i64, C.POINTER(f64)]
    L.mc_reserve.argtypes = [vp, i64]
    L.mc_save_state.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
    L.mc_load_state.argtypes = [vp, vp, C.c_size_t]
    L.mc_set_weights.argtypes = [vp, vp]
    L.mc_apply_gradient.argtypes = [vp, vp, i32, f64]
    L.mc_stream.argtypes = [vp, C.POINTER(vp)]
    L.mc_profile_phases.argtypes = [vp, i64, P(np.float64)]
    L.mc_replay_delivery.argtypes = [vp, i64, i64, vp, i64, C.POINTER(f64), C.POINTER(i64)]
    L.mc_atomic_rate.argtypes = [vp, i64, C.POINTER(f64)]
    L.mc_last_adjoint_ms.argtypes = [vp, C.POINTER(f64), C.POINTER(f64)]
    L.mc_get_persist_shape.argtypes = [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.mc_get_phase_table.argtypes = [vp, vp, i64, C.POINTER(i32)]
    _lib = L
    return L


def _check(rc: int, where: str):
    if rc != MC_OK:
        raise MCError(rc, where, lib().mc_last_error().decode(errors="replace"))


def _arr(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


class Network:
    """An ``mc_net`` handle: build, simulate, observe, differentiate."""

    def __init__(self, w: Workload, host_only: bool = False, stream: Optional[int] = None,
                 device_connect: bool = False, allocator=None):
        """allocator: optional (dev_alloc(bytes) -> device pointer int, dev_free(ptr))
        pair of Python callables; every device buffer of the network comes from it."""
        self.workload = w
        n = w.n_pops
        self._keep = [
            _arr(w.pop_size, np.int32), _arr(np.asarray(w.conn, float).reshape(-1), np.float64),
            _arr(np.asarray(w.w_mean, float).reshape(-1), np.float64), _arr(w.d_mean, np.float64),
            _arr(w.k_ext, np.float64),
        ]
        if w.inst_seed is None:
            scales, seeds = _arr([w.scale], np.float64), _arr([w.seed], np.uint64)
        else:
            scales, seeds = _arr(w.inst_scale, np.float64), _arr(w.inst_seed, np.uint64)
        self._keep += [scales, seeds]
        c = mc_config()
        c.struct_size = C.sizeof(mc_config)
        c.n_pops = n
        c.pop_size = self._keep[0].ctypes.data_as(C.POINTER(C.c_int32))
        c.rule = w.rule
        c.conn = self._keep[1].ctypes.data_as(C.POINTER(C.c_double))
        c.w_mean_pA = self._keep[2].ctypes.data_as(C.POINTER(C.c_double))
        c.w_rel_sd = w.w_rel_sd
        c.d_mean_ms = self._keep[3].ctypes.data_as(C.POINTER(C.c_double))
        c.d_rel_sd = w.d_rel_sd
        c.d_min_steps, c.d_max_steps = w.d_min_steps, w.d_max_steps
        c.k_ext = self._keep[4].ctypes.data_as(C.POINTER(C.c_double))
        c.nu_ext_hz, c.w_ext_pA = w.nu_ext, w.w_ext
        c.tau_m_ms, c.c_m_pF, c.e_l_mV, c.v_reset_mV = w.tau_m, w.c_m, w.e_l, w.v_reset
        c.v_th_mV, c.t_ref_ms, c.tau_syn_ms, c.i_e_pA, c.h_ms = w.v_th, w.t_ref, w.tau_syn, w.i_e, w.h
        c.v0_lo_mV, c.v0_hi_mV = w.v0_lo, w.v0_hi
        c.n_instances = len(seeds)
        c.inst_scale = scales.ctypes.data_as(C.POINTER(C.c_double))
        c.inst_seed = seeds.ctypes.data_as(C.POINTER(C.c_uint64))
        c.hip_stream = stream
        c.flags = (FLAG_HOST_ONLY if host_only else 0) | (FLAG_DEVICE_CONNECT if device_connect else 0)
        if allocator is not None:
            fa, ff = allocator
            # the callbacks must outlive the network: kept on the object
            self._hooks = (DEV_ALLOC_FN(lambda nbytes, ctx: fa(nbytes) or None),
                           DEV_FREE_FN(lambda ptr, ctx: ff(ptr)))
            c.dev_alloc = C.cast(self._hooks[0], C.c_void_p)
            c.dev_free = C.cast(self._hooks[1], C.c_void_p)
        h = C.c_void_p()
        _check(lib().mc_build_network(C.byref(c), C.byref(h)), "mc_build_network")
        self.h = h
        N, M, ni = C.c_int64(), C.c_int64(), C.c_int32()
        _check(lib().mc_get_sizes(self.h, C.byref(N), C.byref(M), C.byref(ni)), "mc_get_sizes")
        self.N, self.M, self.n_instances = N.value, M.value, ni.value
        self.n_pops = n

    def close(self):
        if getattr(self, "h", None):
            lib().mc_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- the simulation calls -------------------------------------------
    def simulate(self, steps: int):
        _check(lib().mc_simulate(self.h, int(steps)), "mc_simulate")

    def simulate_noalloc(self, steps: int):
        """mc_simulate_noalloc: the persistent scheme without any allocation
        (reserve the raster first)."""
        _check(lib().mc_simulate_noalloc(self.h, int(steps)), "mc_simulate_noalloc")

    def spikes(self, begin: int = 0, end: int = 2**31 - 1):
        cnt = C.c_int64()
        rc = lib().mc_get_spikes(self.h, begin, end, None, None, 0, C.byref(cnt))
        if rc not in (MC_OK, MC_ERR_BUFFER_TOO_SMALL):
            _check(rc, "mc_get_spikes")
        s = np.zeros(cnt.value, np.int32)
        i = np.zeros(cnt.value, np.int32)
        _check(lib().mc_get_spikes(self.h, begin, end, s.ctypes.data, i.ctypes.data, cnt.value, C.byref(cnt)),
               "mc_get_spikes")
        return s, i

    def adjoint(self, window: int, ckpt_every: int, v_target: float, fp32: bool, grad_ptr: int,
                input_mode: int = 0) -> float:
        """mc_adjoint; input_mode: ADJ_INPUT_AUTO, ADJ_INPUT_RECORD or ADJ_INPUT_REPLAY."""
        a = mc_adjoint_config()
        a.struct_size = C.sizeof(mc_adjoint_config)
        a.window_steps, a.ckpt_every, a.v_target_mV = window, ckpt_every, v_target
        a.grad_dtype = GRAD_F32 if fp32 else GRAD_F64
        a.input_mode = input_mode
        loss = C.c_double()
        _check(lib().mc_adjoint(self.h, C.byref(a), C.c_void_p(grad_ptr), C.byref(loss)), "mc_adjoint")
        return loss.value

    # --- introspection ----------------------------------------------------
    def synapses(self):
        rp = np.zeros(self.N + 1, np.int64)
        tg = np.zeros(self.M, np.int32)
        w = np.zeros(self.M, np.int32)
        d = np.zeros(self.M, np.uint8)
        _check(lib().mc_get_synapses(self.h, rp.ctypes.data, tg.ctypes.data, w.ctypes.data, d.ctypes.data),
               "mc_get_synapses")
        return rp, tg, w, d

    def state(self):
        y = np.zeros(self.N, np.float64)
        I = np.zeros(self.N, np.float64)
        r = np.zeros(self.N, np.int32)
        _check(lib().mc_get_state(self.h, y.ctypes.data, I.ctypes.data, r.ctypes.data), "mc_get_state")
        return y, I, r

    def set_state(self, y, I, r):
        _check(lib().mc_set_state(self.h, _arr(y, np.float64), _arr(I, np.float64), _arr(r, np.int32)),
               "mc_set_state")

    def ring(self, depth: int = RING_SLOTS) -> np.ndarray:
        out = np.zeros((depth, self.N), np.int64)
        _check(lib().mc_get_ring(self.h, depth, out), "mc_get_ring")
        return out

    def inject(self, k: int, neuron: int, value: int):
        _check(lib().mc_inject(self.h, k, neuron, value), "mc_inject")

    def propagators(self) -> np.ndarray:
        p = np.zeros(4, np.float64)
        _check(lib().mc_get_propagators(self.h, p), "mc_get_propagators")
        return p

    def tables(self) -> np.ndarray:
        t = np.zeros((self.n_pops, 64), np.uint64)
        _check(lib().mc_get_drive_tables(self.h, t), "mc_get_drive_tables")
        return t

    def counters(self):
        c = mc_counters()
        _check(lib().mc_get_counters(self.h, C.byref(c)), "mc_get_counters")
        return {"step": c.step, "spikes": c.spikes, "events": c.events,
                "spikes_per_pop": np.array(c.spikes_per_pop[: self.n_pops], np.int64)}

    def instance_offsets(self) -> np.ndarray:
        o = np.zeros(self.n_instances + 1, np.int64)
        _check(lib().mc_get_instance_offsets(self.h, o), "mc_get_instance_offsets")
        return o

    def pop_offsets(self, instance: int = 0) -> np.ndarray:
        o = np.zeros(self.n_pops + 1, np.int64)
        _check(lib().mc_get_pop_offsets(self.h, instance, o), "mc_get_pop_offsets")
        return o

    def set_launch(self, scheme=SCHEME_STEP_KERNELS, block=256, neurons_per_wg=256, steps_per_graph=1000,
                   rows_per_wave=0):
        l = mc_launch(C.sizeof(mc_launch), scheme, block, neurons_per_wg, steps_per_graph, rows_per_wave)
        _check(lib().mc_set_launch(self.h, C.byref(l)), "mc_set_launch")

    @staticmethod
    def _launch_dict(l) -> dict:
        return {"scheme": l.scheme, "block": l.block, "neurons_per_wg": l.neurons_per_wg,
                "steps_per_graph": l.steps_per_graph, "rows_per_wave": l.rows_per_wave}

    def get_launch(self) -> dict:
        l = mc_launch()
        _check(lib().mc_get_launch(self.h, C.byref(l)), "mc_get_launch")
        return self._launch_dict(l)

    def tune(self, steps: int) -> dict:
        """Times the candidate launch shapes and keeps the fastest (state
        restored); with MC_TUNE_CACHE set, a stored choice is applied untimed."""
        l = mc_launch()
        _check(lib().mc_tune(self.h, steps, C.byref(l)), "mc_tune")
        return self._launch_dict(l)

    def profile_phases(self, steps: int) -> dict:
        us = np.zeros(8, np.float64)
        _check(lib().mc_profile_phases(self.h, steps, us), "mc_profile_phases")
        # deliver: the delay-1 events (LDS window) or every event of the step (buckets);
        # drive_pending: drive of the next step (and pending delivery in the LDS window)
        return dict(zip(["update", "publish", "wait", "gather", "deliver", "total", "drive_pending",
                         "poll"], us.tolist()))

    def phase_table(self) -> np.ndarray:
        """[G, 8] per-workgroup phase times (us/step) of the last profile_phases."""
        g = C.c_int32()
        rc = lib().mc_get_phase_table(self.h, None, 0, C.byref(g))
        if rc not in (MC_OK, MC_ERR_BUFFER_TOO_SMALL):
            _check(rc, "mc_get_phase_table")
        out = np.zeros((g.value, 8), np.float64)
        _check(lib().mc_get_phase_table(self.h, out.ctypes.data, out.size, C.byref(g)), "mc_get_phase_table")
        return out

    def replay_delivery(self, begin: int, end: int, want_ring: bool = False):
        """Delivers the recorded spikes of steps [begin, end) in one launch;
        returns (ms, events, ring or None)."""
        ms, ev = C.c_double(), C.c_int64()
        ring = None
        ptr, cap = None, 0
        if want_ring:
            ring = np.zeros((end - begin + 101, self.N), np.int64)
            ptr, cap = ring.ctypes.data, ring.size
        _check(lib().mc_replay_delivery(self.h, begin, end, ptr, cap, C.byref(ms), C.byref(ev)), "mc_replay_delivery")
        return ms.value, ev.value, ring

    def atomic_rate(self, entries: int) -> float:
        g = C.c_double()
        _check(lib().mc_atomic_rate(self.h, entries, C.byref(g)), "mc_atomic_rate")
        return g.value

    def probe_stream(self, nbytes: int) -> float:
        """Streaming-read bandwidth (GB/s) over nbytes of device memory."""
        g = C.c_double()
        _check(lib().mc_probe_stream(self.h, int(nbytes), C.byref(g)), "mc_probe_stream")
        return g.value

    def probe_atomics(self, slots: int, pattern: int) -> float:
        """int64 atomic adds (1e9/s) into a slots x ring-stride table; pattern
        0 uniform, 1 the delivery's row and delay pattern."""
        g = C.c_double()
        _check(lib().mc_probe_atomics(self.h, int(slots), int(pattern), C.byref(g)), "mc_probe_atomics")
        return g.value

    def probe_exchange(self, steps: int) -> float:
        """us per step of the persistent scheme's exchange alone."""
        g = C.c_double()
        _check(lib().mc_probe_exchange(self.h, int(steps), C.byref(g)), "mc_probe_exchange")
        return g.value

    def last_simulate_ms(self) -> float:
        ms = C.c_double()
        _check(lib().mc_last_simulate_ms(self.h, C.byref(ms)), "mc_last_simulate_ms")
        return ms.value

    def last_kernel_ms(self) -> dict:
        """Persistent kernel launches of the most recent simulate: summed HIP-event
        durations (ms), launches timed and the steps they covered."""
        ms, k, st = C.c_double(), C.c_int64(), C.c_int64()
        _check(lib().mc_last_kernel_ms(self.h, C.byref(ms), C.byref(k), C.byref(st)), "mc_last_kernel_ms")
        return {"ms": ms.value, "launches": k.value, "steps": st.value}

    def persist_shape(self) -> dict:
        """Persistent-scheme shape in use (zeros under the step kernels)."""
        g, b, dl = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().mc_get_persist_shape(self.h, C.byref(g), C.byref(b), C.byref(dl)), "mc_get_persist_shape")
        return {"workgroups": g.value, "targets_per_wg": b.value, "lds_steps": dl.value}

    def last_adjoint_ms(self) -> tuple[float, float]:
        """(forward ms, reverse ms) of the most recent adjoint, from HIP events."""
        f, r = C.c_double(), C.c_double()
        _check(lib().mc_last_adjoint_ms(self.h, C.byref(f), C.byref(r)), "mc_last_adjoint_ms")
        return f.value, r.value

    def reserve(self, steps: int):
        _check(lib().mc_reserve(self.h, steps), "mc_reserve")

    def save_state(self) -> bytes:
        used = C.c_size_t()
        lib().mc_save_state(self.h, None, 0, C.byref(used))
        buf = C.create_string_buffer(used.value)
        _check(lib().mc_save_state(self.h, buf, used.value, C.byref(used)), "mc_save_state")
        return buf.raw

    def load_state(self, blob: bytes):
        _check(lib().mc_load_state(self.h, blob, len(blob)), "mc_load_state")

    def set_weights(self, w_dev_ptr: int):
        _check(lib().mc_set_weights(self.h, C.c_void_p(w_dev_ptr)), "mc_set_weights")

    def apply_gradient(self, grad_dev_ptr: int, fp32: bool, eta: float):
        """mc_apply_gradient: w <- rint((w - eta g) 2^16) 2^-16 pA on the device store."""
        _check(lib().mc_apply_gradient(self.h, C.c_void_p(grad_dev_ptr), GRAD_F32 if fp32 else GRAD_F64, float(eta)),
               "mc_apply_gradient")

    def stream(self) -> int:
        s = C.c_void_p()
        _check(lib().mc_stream(self.h, C.byref(s)), "mc_stream")
        return s.value or 0
