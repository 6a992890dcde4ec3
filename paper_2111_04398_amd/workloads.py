"""Workload presets: parameter values of the synthetic networks, nothing else.

This module holds no arithmetic of the method.  It is the one module shared by
the product binding, the tests and the benchmark (and, through plain dicts,
the CPU oracle): every quantity that the simulation derives from these values
(population scaling, propagators, Poisson tables, quantised weights, the
network itself) is computed separately by the library and by the oracle.

The paper (Methods, Supplementary Fig. 1 caption) fixes the time grid
h = 0.1 ms, the smallest delay 0.1 ms, tau_syn = 0.5 ms and tau_m = 10 ms, and
identifies the workload as the Potjans-Diesmann cortical microcircuit of about
80,000 neurons and 3e8 synapses (Fig. 1a caption).  The published connection
table, external in-degrees and "optimized initial conditions" are not in the
paper; the synthetic stand-ins below keep the published population sizes and
the shape of the table (values 0-0.37, same-layer E/I entries of a few
percent to a few tens of percent).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

RULE_FIXED_INDEGREE = 0
RULE_BERNOULLI = 1

#: Population names and sizes of the full-scale microcircuit (Fig. 1a caption:
#: four layers, one excitatory and one inhibitory population each).
MICROCIRCUIT_POPS = ["L23E", "L23I", "L4E", "L4I", "L5E", "L5I", "L6E", "L6I"]
MICROCIRCUIT_SIZES = [20683, 5834, 21915, 5479, 4850, 1065, 14395, 2948]

#: Synthetic connection probabilities p[post][pre] (rows: target population,
#: columns: source population), same population order as above.
MICROCIRCUIT_P = [
    [0.100, 0.111, 0.060, 0.060, 0.020, 0.000, 0.010, 0.000],
    [0.130, 0.134, 0.040, 0.020, 0.010, 0.000, 0.010, 0.000],
    [0.010, 0.010, 0.080, 0.138, 0.010, 0.000, 0.040, 0.000],
    [0.030, 0.000, 0.100, 0.193, 0.010, 0.000, 0.080, 0.000],
    [0.080, 0.060, 0.020, 0.000, 0.060, 0.370, 0.020, 0.000],
    [0.050, 0.020, 0.010, 0.000, 0.070, 0.370, 0.010, 0.000],
    [0.020, 0.000, 0.040, 0.030, 0.020, 0.020, 0.060, 0.289],
    [0.010, 0.000, 0.010, 0.000, 0.020, 0.000, 0.090, 0.357],
]

J_PA = 87.8          # excitatory mean weight, pA
G_REL = 4.0          # inhibitory weight = -G_REL * J


@dataclass
class Workload:
    name: str
    n_pops: int
    pop_size: List[int]
    pop_is_exc: List[int]
    rule: int
    conn: List[List[float]]        # [post][pre]: in-degree (fixed) or probability
    w_mean: List[List[float]]      # [post][pre], pA, signed
    d_mean: List[float]            # per presynaptic population, ms
    k_ext: List[float]             # external in-degree per population
    w_rel_sd: float = 0.1
    d_rel_sd: float = 0.5
    d_min_steps: int = 1
    d_max_steps: int = 100
    nu_ext: float = 8.0            # Hz
    w_ext: float = J_PA            # pA
    tau_m: float = 10.0
    c_m: float = 250.0
    e_l: float = -65.0
    v_reset: float = -65.0
    v_th: float = -50.0
    t_ref: float = 2.0
    tau_syn: float = 0.5
    i_e: float = 0.0
    h: float = 0.1
    v0_lo: float = -65.0
    v0_hi: float = -50.0
    seed: int = 1
    scale: float = 1.0
    # batched form: per-instance scales and seeds (None: one instance)
    inst_scale: Optional[List[float]] = None
    inst_seed: Optional[List[int]] = None
    # protocol
    presim_steps: int = 1000
    sim_steps: int = 10000
    # adjoint
    adj_window: int = 0
    adj_ckpt_every: int = 0
    adj_v_target: float = -58.0
    adj_fp32: bool = False

    def to_dict(self) -> dict:
        return dataclasses.asdict(self)

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    def instance(self, b: int) -> "Workload":
        """The standalone single-instance workload of batched instance b."""
        if self.inst_seed is None:
            return self.replace()
        return self.replace(name=f"{self.name}[{b}]", seed=int(self.inst_seed[b]),
                            scale=float(self.inst_scale[b]), inst_scale=None, inst_seed=None)


def balanced(seed: int = 1) -> Workload:
    """Balanced random network: 4000 E + 1000 I, fixed in-degree 400 E + 100 I
    drawn with replacement, E weight J, I weight -4J, Poisson drive of 1000
    inputs at 8 Hz with weight J; 1 s of model time after a 0.1 s presim."""
    n = 2
    return Workload(
        name="balanced_5k", n_pops=n, pop_size=[4000, 1000], pop_is_exc=[1, 0],
        rule=RULE_FIXED_INDEGREE,
        conn=[[400.0, 100.0], [400.0, 100.0]],
        w_mean=[[J_PA, -G_REL * J_PA], [J_PA, -G_REL * J_PA]],
        d_mean=[1.5, 0.75], k_ext=[1000.0, 1000.0], seed=seed,
        presim_steps=1000, sim_steps=10000)


def microcircuit(seed: int = 1, scale: float = 1.0, sim_steps: int = 100000) -> Workload:
    """Full-scale microcircuit shape: 8 populations, 77,169 neurons, pairwise
    Bernoulli connectivity from the synthetic table, L4E->L2/3E weight 2J,
    external in-degrees 1500 + 200*index, 10 s after a 0.1 s presim."""
    n = 8
    exc = [1, 0] * 4
    w = [[(J_PA if exc[b] else -G_REL * J_PA) for b in range(n)] for a in range(n)]
    w[0][2] = 2.0 * J_PA
    return Workload(
        name="microcircuit" if scale == 1.0 else f"microcircuit_x{scale:g}",
        n_pops=n, pop_size=list(MICROCIRCUIT_SIZES), pop_is_exc=exc,
        rule=RULE_BERNOULLI, conn=[list(r) for r in MICROCIRCUIT_P], w_mean=w,
        d_mean=[1.5 if exc[b] else 0.75 for b in range(n)],
        k_ext=[1500.0 + 200.0 * k for k in range(n)], seed=seed, scale=scale,
        presim_steps=1000, sim_steps=sim_steps)


def batch_scales(n_instances: int = 64) -> List[float]:
    """Instance scales 0.05 + 0.20*u, u the 53-bit uniform from word 0 of the
    Philox4x64-10 block with counter (b, 0, 0, 7) and key (1, 0); numpy's
    Philox pre-increments its counter, hence the counter b - 1 (with borrow)."""
    out = []
    m64 = (1 << 64) - 1
    for b in range(n_instances):
        c = ((7 << 192) | b) - 1          # 256-bit counter, word 0 least significant
        ctr = [(c >> (64 * k)) & m64 for k in range(4)]
        bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64), key=np.array([1, 0], dtype=np.uint64))
        w0 = int(bg.random_raw(4)[0])
        out.append(0.05 + 0.20 * ((w0 >> 11) * 2.0 ** -53))
    return out


def batched(n_instances: int = 64, sim_steps: int = 20000) -> Workload:
    """64 microcircuit instances of uneven size (scale in [0.05, 0.25] of the
    full population sizes, connection probabilities kept so in-degrees scale
    with the instance, external drive unscaled), seeds 1001.. ; 2 s each."""
    base = microcircuit(seed=1001)
    return base.replace(name=f"batched_{n_instances}", inst_scale=batch_scales(n_instances),
                        inst_seed=[1001 + b for b in range(n_instances)], sim_steps=sim_steps)


def adjoint_small() -> Workload:
    """Adjoint at scale 0.1 of the microcircuit (7,717 neurons): 2000-step
    window from a fresh network, loss vs -58 mV, checkpoint every 200 steps,
    FP64 gradient."""
    return microcircuit(seed=1, scale=0.1).replace(
        name="adjoint_x0.1", presim_steps=0, sim_steps=2000,
        adj_window=2000, adj_ckpt_every=200, adj_v_target=-58.0, adj_fp32=False)


def adjoint_full() -> Workload:
    """Full-scale adjoint: 2000-step window, checkpoint every 100 steps, FP32
    per-synapse gradient accumulated from FP64 adjoint states."""
    return microcircuit(seed=1).replace(
        name="adjoint_full", presim_steps=0, sim_steps=2000,
        adj_window=2000, adj_ckpt_every=100, adj_v_target=-58.0, adj_fp32=True)


PRESETS = {
    "balanced": balanced,
    "microcircuit": microcircuit,
    "batched": batched,
    "adjoint_small": adjoint_small,
    "adjoint_full": adjoint_full,
}
