"""Pins of the oracle's simulation step: closed-form responses of the
exact-integration LIF neuron, and brute-force equality on tiny networks."""
import math

import mpmath
import numpy as np
import pytest

import oracle
from naive_sim import Naive
from paper_2111_04398_amd import workloads
from test_oracle_builder import tiny_bernoulli, tiny_fixed

mpmath.mp.dps = 40


def lone_neuron(i_e=0.0):
    """One neuron, no synapses, no drive (lambda = 0), V0 = E_L."""
    w = workloads.balanced()
    return w.replace(n_pops=1, pop_size=[1], pop_is_exc=[1], conn=[[0.0]], w_mean=[[87.8]], d_mean=[1.5],
                     k_ext=[0.0], v0_lo=-65.0, v0_hi=-65.0, i_e=i_e)


def trajectory(o, steps):
    ys = []
    for _ in range(steps):
        o.run(1)
        ys.append(o.state()[0][0])
    return np.array(ys)


@pytest.mark.parametrize("wq", [5754061, -4 * 5754061, 1])
def test_single_input_response_closed_form(wq):
    """A current jump w read at step n enters I at the end of step n, so the
    membrane response at the post-state of step n+k is
    y = tau_s tau_m / (C (tau_m - tau_s)) w (e^{-k h/tau_m} - e^{-k h/tau_s})
    (the exact solution, evaluated with 40-digit exponentials).  Rounding
    grows at most linearly in k: tolerance 8 ulp * (k+1) relative."""
    o = oracle.Oracle(lone_neuron().to_dict())
    o.inject(0, 0, wq)
    ys = trajectory(o, 400)
    w = mpmath.mpf(wq) / 65536
    A = mpmath.mpf("0.5") * 10 / (250 * mpmath.mpf("9.5"))
    for k in range(400):
        exact = A * w * (mpmath.exp(-mpmath.mpf(k) / 100) - mpmath.exp(-mpmath.mpf(k) / 5))
        if k == 0:
            assert ys[0] == 0.0
            continue
        rel = abs((mpmath.mpf(ys[k]) - exact) / exact)
        assert rel <= 8 * (k + 1) * 2.0**-53, (k, float(rel))
    if wq == 5754061:
        k = int(np.argmax(ys))
        assert k == 16 and abs(ys[k] - 0.1499775) < 1e-7


def test_dc_steady_state():
    """Constant current I_e = 300 pA below rheobase (375 pA): y_n equals the
    exact R I_e (1 - e^{-n h/tau_m}) within 1e-12 mV, and reaches 12 mV within
    1e-12 after 6000 steps."""
    o = oracle.Oracle(lone_neuron(i_e=300.0).to_dict())
    ys = trajectory(o, 6000)
    for n in (1, 10, 100, 1000, 3000, 5999):
        exact = 12 * (1 - mpmath.exp(-mpmath.mpf(n + 1) / 100))
        assert abs(ys[n] - float(exact)) < 1e-12
    assert abs(ys[-1] - 12.0) <= 1e-12
    assert o.raster()[0].size == 0


@pytest.mark.parametrize("ie,first,isi", [(400.0, 277, 298), (500.0, 138, 159), (1000.0, 47, 68)])
def test_dc_periodic_firing(ie, first, isi):
    """Suprathreshold DC from rest: y_{n+1} = R I_e (1 - e^{-(n+1)h/tau_m}); the
    first spike is at step k-1, k = ceil(ln(1 - 15/(R I_e)) / (-h/tau_m)), and
    after a reset and 20 refractory steps the cycle repeats: ISI = 20 + k.
    The printed step numbers are recomputed here in 40 digits."""
    R = mpmath.mpf(10) / 250
    k = int(mpmath.ceil(mpmath.log(1 - 15 / (R * ie)) / (-mpmath.mpf(1) / 100)))
    assert (k - 1, 20 + k) == (first, isi)
    o = oracle.Oracle(lone_neuron(i_e=ie).to_dict())
    o.run(first + 5 * isi + 1)
    s, _ = o.raster()
    assert list(s) == [first + q * isi for q in range(6)]


def test_refractory_clamp():
    """After a spike at step n, y stays at the reset value for exactly 20
    steps (t_ref / h) while I keeps integrating."""
    o = oracle.Oracle(lone_neuron(i_e=1000.0).to_dict())
    o.run(48)
    assert list(o.raster()[0]) == [47]
    for k in range(20):
        o.inject(0, 0, 65536 * 100)
        o.run(1)
        y, I, r = o.state()
        assert y[0] == 0.0 and r[0] == 19 - k
        assert I[0] > 0
    o.run(1)
    assert o.state()[0][0] > 0.0


@pytest.mark.parametrize("mk,steps", [(tiny_fixed, 2000), (tiny_bernoulli, 1500)])
def test_brute_force_tiny_networks(mk, steps):
    """Tiny networks: the oracle and the brute-force event-list simulator give
    identical rasters, state bits, pending inputs and event counts; events =
    sum of the out-degrees of all spikes."""
    w = mk().to_dict()
    o = oracle.Oracle(w)
    nv = Naive(w)
    o.run(steps)
    nv.run(steps)
    s, i = o.raster()
    assert len(s) > 50
    assert list(zip(s.tolist(), i.tolist())) == nv.raster
    y, I, r = o.state()
    assert np.array_equal(y.view(np.uint64), np.array(nv.y).view(np.uint64))
    assert np.array_equal(I.view(np.uint64), np.array(nv.I).view(np.uint64))
    assert np.array_equal(r, np.array(nv.r))
    assert np.array_equal(o.ring(128), nv.logical_ring(128))
    sp, ev = o.counters()
    rp = o.synapses()[0]
    assert ev == nv.events == int(np.diff(rp)[i].sum())


def test_thread_count_invariance():
    """One OpenMP thread and all threads give bit-identical runs."""
    w = workloads.balanced().to_dict()
    res = []
    for t in (1, 8):
        oracle.set_threads(t)
        o = oracle.Oracle(w)
        o.run(300)
        res.append((o.raster(), o.state(), o.ring(128)))
    oracle.set_threads(8)
    (a, b) = res
    assert np.array_equal(a[0][0], b[0][0]) and np.array_equal(a[0][1], b[0][1])
    for x, y in zip(a[1], b[1]):
        assert np.array_equal(x, y)
    assert np.array_equal(a[2], b[2])


def test_balanced_activity_sanity():
    """Not parity: the balanced network fires asynchronously at a few tens of
    Hz (no silent or saturated population)."""
    o = oracle.Oracle(workloads.balanced().to_dict())
    o.run(2000)
    sp, ev = o.counters()
    rates = sp / np.array([4000, 1000]) / 0.2
    assert np.all(rates > 5) and np.all(rates < 100)
