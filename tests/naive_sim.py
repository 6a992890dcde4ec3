"""Brute-force reference for tiny networks, in plain Python.

An independent, deliberately naive implementation of the same specification
as the CPU oracle: it draws every random number through numpy's own
Philox4x64-10 bit generator (not the oracle's), builds the synapse list by
enumerating pairs/slots, and simulates with a dictionary of pending
(step, target) -> integer input instead of a ring buffer.  Floating-point
expressions are evaluated with Python floats (IEEE double, no contraction), in
the order the specification fixes.  Only usable for tens of neurons.
"""
from __future__ import annotations

import math
from collections import defaultdict

import numpy as np

M64 = (1 << 64) - 1
TAG_V0, TAG_CONN, TAG_SRC, TAG_W, TAG_D, TAG_DRIVE = 1, 2, 3, 4, 5, 6


def philox_np(c0: int, c1: int, c2: int, c3: int, k0: int, k1: int = 0):
    """Philox4x64-10 block for counter (c0..c3), key (k0, k1) via numpy; numpy
    increments its 256-bit counter before generating, so it is given C - 1."""
    c = (c0 | (c1 << 64) | (c2 << 128) | (c3 << 192)) - 1
    c %= 1 << 256
    ctr = np.array([(c >> (64 * k)) & M64 for k in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=ctr, key=np.array([k0, k1], dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


def u53(w):
    return (w >> 11) * 2.0 ** -53


def normal(a, b, tag, seed):
    w = philox_np(a, b, 0, tag, seed)
    u1 = ((w[0] >> 11) + 1) * 2.0 ** -53
    u2 = (w[1] >> 11) * 2.0 ** -53
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(6.283185307179586 * u2)


class Naive:
    def __init__(self, p: dict):
        self.p = p
        n = p["n_pops"]
        sizes = [max(1, int(np.rint(p.get("scale", 1.0) * s))) for s in p["pop_size"]]
        self.off = [0]
        for s in sizes:
            self.off.append(self.off[-1] + s)
        self.N = self.off[-1]
        self.pop = []
        for a in range(n):
            self.pop += [a] * sizes[a]
        h = p["h"]
        self.P22 = math.exp(-h / p["tau_m"])
        self.P11 = math.exp(-h / p["tau_syn"])
        self.P21 = ((p["tau_syn"] * p["tau_m"]) / (p["c_m"] * (p["tau_m"] - p["tau_syn"]))) * (self.P22 - self.P11)
        self.P20 = -(p["tau_m"] / p["c_m"]) * math.expm1(-h / p["tau_m"])
        self.jq = int(np.rint(p["w_ext"] * 65536.0))
        self.ref = int(np.rint(p["t_ref"] / h))
        self.theta = p["v_th"] - p["e_l"]
        self.yreset = p["v_reset"] - p["e_l"]
        self.tables = []
        for a in range(n):
            lam = ((p["nu_ext"] * p["k_ext"][a]) * h) * 1e-3
            pk = math.exp(-lam)
            F = pk
            T = []
            for k in range(64):
                if k > 0:
                    pk = pk * lam / k
                    F = F + pk
                T.append(min(int(math.floor(F * 4294967296.0)), 1 << 32))
            T[63] = 1 << 32
            self.tables.append(T)
        self.synapses = self._build()
        self.y = []
        for i in range(self.N):
            w = philox_np(i >> 2, 0, 0, TAG_V0, p["seed"])
            self.y.append((p["v0_hi"] - p["v0_lo"]) * u53(w[i & 3]) + (p["v0_lo"] - p["e_l"]))
        self.I = [0.0] * self.N
        self.r = [0] * self.N
        self.pending = defaultdict(int)
        self.step = 0
        self.raster = []
        self.events = 0

    def _wd(self, a, b, post, pre):
        p = self.p
        mu = p["w_mean"][post][pre]
        z = normal(a, b, TAG_W, p["seed"])
        w = mu + (p["w_rel_sd"] * abs(mu)) * z
        wq = int(np.rint(w * 65536.0))
        md = p["d_mean"][pre]
        z = normal(a, b, TAG_D, p["seed"])
        d = int(np.rint((md + (p["d_rel_sd"] * md) * z) / p["h"]))
        d = min(max(d, p["d_min_steps"]), p["d_max_steps"])
        return wq, d

    def _build(self):
        """List of (source, target, slot, w_q, delay) in canonical order."""
        p = self.p
        n = p["n_pops"]
        syn = []
        if p["rule"] == 0:
            for j in range(self.N):
                a = self.pop[j]
                m = 0
                for b in range(n):
                    Nb = self.off[b + 1] - self.off[b]
                    for _ in range(int(round(p["conn"][a][b]))):
                        w = philox_np(j, m >> 2, 0, TAG_SRC, p["seed"])
                        src = self.off[b] + (((w[m & 3] >> 32) * Nb) >> 32)
                        wq, d = self._wd(j, m, a, b)
                        syn.append((src, j, m, wq, d))
                        m += 1
        else:
            for i in range(self.N):
                b = self.pop[i]
                for j in range(self.N):
                    a = self.pop[j]
                    T = int(math.floor(p["conn"][a][b] * 4294967296.0))
                    w = philox_np(i, j >> 2, 0, TAG_CONN, p["seed"])
                    if (w[j & 3] >> 32) < T:
                        wq, d = self._wd(i, j, a, b)
                        syn.append((i, j, 0, wq, d))
        syn.sort(key=lambda s: (s[0], s[1], s[2]))
        return syn

    def csr(self):
        rp = np.zeros(self.N + 1, np.int64)
        for s in self.synapses:
            rp[s[0] + 1] += 1
        rp = np.cumsum(rp)
        tg = np.array([s[1] for s in self.synapses], np.int32)
        w = np.array([s[3] for s in self.synapses], np.int32)
        d = np.array([s[4] for s in self.synapses], np.uint8)
        return rp, tg, w, d

    def run(self, steps):
        p = self.p
        rows = defaultdict(list)
        for s in self.synapses:
            rows[s[0]].append(s)
        for _ in range(steps):
            n = self.step
            spikes = []
            blocks = {}
            for i in range(self.N):
                q = i >> 2
                if q not in blocks:
                    blocks[q] = philox_np(n, q, 0, TAG_DRIVE, p["seed"])
                u = blocks[q][i & 3] >> 32
                T = self.tables[self.pop[i]]
                k = 0
                while u >= T[k]:
                    k += 1
                x_int = self.pending.pop((n, i), 0) + k * self.jq
                x = float(x_int) * 2.0 ** -16
                free = self.r[i] == 0
                if free:
                    y = self.P22 * self.y[i] + self.P21 * self.I[i]
                    if p["i_e"] != 0.0:
                        y = y + self.P20 * p["i_e"]
                    self.y[i] = y
                else:
                    self.r[i] -= 1
                self.I[i] = self.P11 * self.I[i] + x
                if free and self.y[i] >= self.theta:
                    spikes.append(i)
                    self.y[i] = self.yreset
                    self.r[i] = self.ref
            for i in spikes:
                self.raster.append((n, i))
                for s in rows[i]:
                    self.pending[(n + s[4], s[1])] += s[3]
                self.events += len(rows[i])
            self.step += 1

    def logical_ring(self, depth=128):
        out = np.zeros((depth, self.N), np.int64)
        for (n, i), v in self.pending.items():
            k = n - self.step
            if 0 <= k < depth:
                out[k, i] += v
        return out
