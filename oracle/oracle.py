"""ctypes front end of the CPU oracle (``mc_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the product package.  It takes a
plain ``dict`` of workload parameters (the keys of
``paper_2111_04398_amd.workloads.Workload.to_dict``) so that it needs nothing
from the product package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mc_oracle.cpp")
_LIB = os.path.join(_HERE, "libmc_oracle.so")
MAXPOP = 16


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (IEEE double, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", _SRC, "-o", _LIB + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("n_pops", C.c_int32),
        ("pop_size", C.c_int32 * MAXPOP),
        ("pop_is_exc", C.c_int32 * MAXPOP),
        ("rule", C.c_int32),
        ("conn", C.c_double * (MAXPOP * MAXPOP)),
        ("w_mean", C.c_double * (MAXPOP * MAXPOP)),
        ("w_rel_sd", C.c_double),
        ("d_mean", C.c_double * MAXPOP),
        ("d_rel_sd", C.c_double),
        ("d_min_steps", C.c_int32),
        ("d_max_steps", C.c_int32),
        ("k_ext", C.c_double * MAXPOP),
        ("nu_ext", C.c_double),
        ("w_ext", C.c_double),
        ("tau_m", C.c_double), ("c_m", C.c_double), ("e_l", C.c_double), ("v_reset", C.c_double),
        ("v_th", C.c_double), ("t_ref", C.c_double), ("tau_syn", C.c_double), ("i_e", C.c_double),
        ("h", C.c_double),
        ("v0_lo", C.c_double), ("v0_hi", C.c_double),
        ("seed", C.c_uint64),
        ("scale", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        vp, i64, f64 = C.c_void_p, C.c_int64, C.c_double
        P = np.ctypeslib.ndpointer
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_philox.argtypes = [P(np.uint64), P(np.uint64), P(np.uint64)]
        L.orc_philox_many.argtypes = [i64, P(np.uint64), P(np.uint64), P(np.uint64)]
        L.orc_box_muller.argtypes = [P(np.uint64)]
        L.orc_box_muller.restype = f64
        L.orc_instance_scale.argtypes = [i64]
        L.orc_instance_scale.restype = f64
        L.orc_build.argtypes = [C.POINTER(_Cfg)]
        L.orc_build.restype = vp
        L.orc_build_params.argtypes = [C.POINTER(_Cfg)]
        L.orc_build_params.restype = vp
        L.orc_free.argtypes = [vp]
        L.orc_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i64)]
        L.orc_pop_offsets.argtypes = [vp, P(np.int64)]
        L.orc_synapses.argtypes = [vp, P(np.int64), P(np.int32), P(np.int32), P(np.uint8)]
        L.orc_bernoulli_row.argtypes = [vp, i64, P(np.int32), i64]
        L.orc_bernoulli_row.restype = i64
        L.orc_weight_delay.argtypes = [vp, C.c_uint64, C.c_uint64, C.c_int, C.c_int,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_uint8)]
        L.orc_weight_delay.restype = C.c_int
        L.orc_propagators.argtypes = [vp, P(np.float64)]
        L.orc_tables.argtypes = [vp, P(np.uint64)]
        L.orc_jext_q.argtypes = [vp]
        L.orc_jext_q.restype = i64
        L.orc_poisson_count.argtypes = [vp, i64, i64]
        L.orc_poisson_count.restype = C.c_int
        L.orc_run.argtypes = [vp, i64]
        L.orc_run.restype = f64
        L.orc_step.argtypes = [vp]
        L.orc_step.restype = i64
        L.orc_state.argtypes = [vp, P(np.float64), P(np.float64), P(np.int32)]
        L.orc_set_state.argtypes = [vp, P(np.float64), P(np.float64), P(np.int32)]
        L.orc_ring.argtypes = [vp, i64, P(np.int64)]
        L.orc_inject.argtypes = [vp, i64, i64, i64]
        L.orc_raster_count.argtypes = [vp]
        L.orc_raster_count.restype = i64
        L.orc_raster.argtypes = [vp, P(np.int32), P(np.int32)]
        L.orc_counters.argtypes = [vp, P(np.int64), C.POINTER(i64)]
        L.orc_adjoint.argtypes = [vp, i64, f64, C.c_int, vp, C.POINTER(f64)]
        L.orc_adjoint.restype = C.c_int
        L.orc_fd.argtypes = [vp, i64, f64, f64, P(np.int64), i64, P(np.float64)]
        L.orc_fd.restype = C.c_int
        L.orc_trace.argtypes = [vp, i64, i64, P(np.uint8), P(np.int64), P(np.float64)]
        L.orc_trace.restype = C.c_int
        L.orc_apply_gradient.argtypes = [vp, vp, C.c_int, f64]
        L.orc_apply_gradient.restype = C.c_int
        L.orc_reset.argtypes = [vp]
        L.orc_reset.restype = None
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def philox(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint64)
    lib().orc_philox(np.ascontiguousarray(ctr, np.uint64), np.ascontiguousarray(key, np.uint64), out)
    return out


def philox_many(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = np.ascontiguousarray(ctr, np.uint64).reshape(-1, 4)
    key = np.ascontiguousarray(key, np.uint64).reshape(-1, 2)
    out = np.zeros_like(ctr)
    lib().orc_philox_many(ctr.shape[0], ctr, key, out)
    return out


def box_muller(words) -> float:
    return lib().orc_box_muller(np.ascontiguousarray(words, np.uint64))


def instance_scale(b: int) -> float:
    return lib().orc_instance_scale(b)


def make_cfg(p: dict) -> _Cfg:
    c = _Cfg()
    n = int(p["n_pops"])
    c.n_pops = n
    for a in range(n):
        c.pop_size[a] = int(p["pop_size"][a])
        c.pop_is_exc[a] = int(p["pop_is_exc"][a])
        c.d_mean[a] = float(p["d_mean"][a])
        c.k_ext[a] = float(p["k_ext"][a])
        for b in range(n):
            c.conn[a * n + b] = float(p["conn"][a][b])
            c.w_mean[a * n + b] = float(p["w_mean"][a][b])
    c.rule = int(p["rule"])
    c.w_rel_sd = float(p["w_rel_sd"])
    c.d_rel_sd = float(p["d_rel_sd"])
    c.d_min_steps = int(p["d_min_steps"])
    c.d_max_steps = int(p["d_max_steps"])
    c.nu_ext = float(p["nu_ext"])
    c.w_ext = float(p["w_ext"])
    for k in ("tau_m", "c_m", "e_l", "v_reset", "v_th", "t_ref", "tau_syn", "i_e", "h", "v0_lo", "v0_hi"):
        setattr(c, k, float(p[k]))
    c.seed = int(p["seed"])
    c.scale = float(p.get("scale", 1.0))
    return c


class Oracle:
    """One network instance, built and simulated on the CPU."""

    def __init__(self, params: dict, synapses: bool = True):
        self.params = dict(params)
        self._cfg = make_cfg(params)
        L = lib()
        self.h = L.orc_build(C.byref(self._cfg)) if synapses else L.orc_build_params(C.byref(self._cfg))
        if not self.h:
            raise ValueError("oracle: invalid configuration or weight out of range")
        N, M = C.c_int64(), C.c_int64()
        L.orc_sizes(self.h, C.byref(N), C.byref(M))
        self.N, self.M = N.value, M.value
        self.n_pops = int(params["n_pops"])

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def pop_offsets(self) -> np.ndarray:
        o = np.zeros(self.n_pops + 1, np.int64)
        lib().orc_pop_offsets(self.h, o)
        return o

    def synapses(self):
        rp = np.zeros(self.N + 1, np.int64)
        tg = np.zeros(self.M, np.int32)
        w = np.zeros(self.M, np.int32)
        d = np.zeros(self.M, np.uint8)
        lib().orc_synapses(self.h, rp, tg, w, d)
        return rp, tg, w, d

    def bernoulli_row(self, i: int) -> np.ndarray:
        cap = self.N
        out = np.zeros(cap, np.int32)
        n = lib().orc_bernoulli_row(self.h, i, out, cap)
        return out[:n].copy()

    def weight_delay(self, a: int, b: int, post: int, pre: int):
        w, d = C.c_int32(), C.c_uint8()
        rc = lib().orc_weight_delay(self.h, a, b, post, pre, C.byref(w), C.byref(d))
        if rc != 0:
            raise ValueError("weight out of range")
        return w.value, d.value

    def propagators(self) -> np.ndarray:
        p = np.zeros(4, np.float64)
        lib().orc_propagators(self.h, p)
        return p  # P11, P21, P22, P20

    def tables(self) -> np.ndarray:
        T = np.zeros((self.n_pops, 64), np.uint64)
        lib().orc_tables(self.h, T)
        return T

    def jext_q(self) -> int:
        return lib().orc_jext_q(self.h)

    def poisson_count(self, step: int, i: int) -> int:
        return lib().orc_poisson_count(self.h, step, i)

    def run(self, steps: int) -> float:
        return lib().orc_run(self.h, int(steps))

    @property
    def step(self) -> int:
        return lib().orc_step(self.h)

    def state(self):
        y = np.zeros(self.N, np.float64)
        I = np.zeros(self.N, np.float64)
        r = np.zeros(self.N, np.int32)
        lib().orc_state(self.h, y, I, r)
        return y, I, r

    def set_state(self, y, I, r):
        lib().orc_set_state(self.h, np.ascontiguousarray(y, np.float64), np.ascontiguousarray(I, np.float64),
                            np.ascontiguousarray(r, np.int32))

    def ring(self, depth: int = 128) -> np.ndarray:
        out = np.zeros((depth, self.N), np.int64)
        lib().orc_ring(self.h, depth, out)
        return out

    def inject(self, k: int, i: int, value: int):
        lib().orc_inject(self.h, k, i, value)

    def raster(self):
        n = lib().orc_raster_count(self.h)
        s = np.zeros(n, np.int32)
        i = np.zeros(n, np.int32)
        if n:
            lib().orc_raster(self.h, s, i)
        return s, i

    def counters(self):
        sp = np.zeros(self.n_pops, np.int64)
        ev = C.c_int64()
        lib().orc_counters(self.h, sp, C.byref(ev))
        return sp, ev.value

    def adjoint(self, S: int, y_star_rel: float, fp32: bool = False):
        """Loss and dL/dw (pA) over the S steps from the current step, spikes
        frozen; the state there, pending input included, is held fixed.  The
        network advances by S steps."""
        g = np.zeros(self.M, np.float32 if fp32 else np.float64)
        loss = C.c_double()
        rc = lib().orc_adjoint(self.h, S, y_star_rel, 1 if fp32 else 0, g.ctypes.data_as(C.c_void_p), C.byref(loss))
        if rc != 0:
            raise RuntimeError("oracle adjoint failed")
        return loss.value, g

    def fd(self, S: int, y_star_rel: float, eps: float, syn) -> np.ndarray:
        """Quad-precision central differences of the same loss (same window)
        for the synapses `syn`."""
        syn = np.ascontiguousarray(syn, np.int64)
        out = np.zeros(len(syn), np.float64)
        rc = lib().orc_fd(self.h, S, y_star_rel, eps, syn, len(syn), out)
        if rc != 0:
            raise RuntimeError("oracle fd failed")
        return out

    def apply_gradient(self, g: np.ndarray, eta: float) -> bool:
        """One gradient-descent step on the stored weights, w <- w - eta g
        (pA), stored again in 2^-16 pA with ties to even; g float64 or
        float32 of M elements.  False (weights unchanged) if a new weight
        would not be finite or would not fit int32."""
        if g.dtype not in (np.float64, np.float32) or g.shape != (self.M,):
            raise ValueError("gradient must be float64 or float32 of M elements")
        g = np.ascontiguousarray(g)
        return lib().orc_apply_gradient(self.h, g.ctypes.data_as(C.c_void_p), 1 if g.dtype == np.float32 else 0,
                                        float(eta)) == 0

    def reset(self):
        """Back to the initial state (step 0), keeping the current weights."""
        lib().orc_reset(self.h)

    def trace(self, S: int, i: int):
        t = np.zeros(S, np.uint8)
        x = np.zeros(S, np.int64)
        y = np.zeros(S + 1, np.float64)
        rc = lib().orc_trace(self.h, S, i, t, x, y)
        if rc != 0:
            raise RuntimeError("oracle trace failed")
        return t, x, y
