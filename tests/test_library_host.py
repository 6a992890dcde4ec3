"""CPU tests of libmc's host side: symbol exports, configuration checks, and
byte equality of the host-built network with the oracle's (no GPU calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2111_04398_amd import mc, workloads
from test_oracle_builder import tiny_bernoulli, tiny_fixed

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    """libmc.so loads and exports every function include/mc.h declares."""
    hdr = open(os.path.join(ROOT, "include", "mc.h")).read()
    declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(mc_\w+)\s*\(", hdr, re.M))
    assert declared == set(mc.EXPORTS)
    L = mc.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert L.mc_abi_version() == 1


@pytest.mark.parametrize("mk", [workloads.balanced, tiny_fixed, tiny_bernoulli,
                                lambda: workloads.microcircuit(scale=0.1)])
def test_host_network_equals_oracle(mk):
    """The library's host builder (independent code) produces the oracle's
    synapse store byte for byte, and the same propagators and tables."""
    w = mk()
    net = mc.Network(w, host_only=True)
    o = oracle.Oracle(w.to_dict())
    assert (net.N, net.M) == (o.N, o.M)
    for a, b in zip(net.synapses(), o.synapses()):
        assert np.array_equal(a, b)
    assert np.array_equal(net.propagators().view(np.uint64), o.propagators().view(np.uint64))
    assert np.array_equal(net.tables(), o.tables())
    assert np.array_equal(net.pop_offsets(0), o.pop_offsets())


def test_batched_instances_equal_standalone_oracle():
    """Instance b of a batched build is the oracle's standalone network with
    that instance's seed and scale, shifted by the instance offset."""
    base = workloads.microcircuit()
    scales = [0.004, 0.006, 0.005]
    w = base.replace(inst_scale=scales, inst_seed=[1001, 1002, 1003])
    net = mc.Network(w, host_only=True)
    rp, tg, wq, d = net.synapses()
    off = net.instance_offsets()
    for b in range(3):
        o = oracle.Oracle(w.instance(b).to_dict())
        orp, otg, owq, od = o.synapses()
        r0, r1 = rp[off[b]], rp[off[b + 1]]
        assert np.array_equal(rp[off[b]:off[b + 1] + 1] - r0, orp)
        assert np.array_equal(tg[r0:r1] - off[b], otg)
        assert np.array_equal(wq[r0:r1], owq)
        assert np.array_equal(d[r0:r1], od)


@pytest.mark.parametrize("change,code", [
    (dict(tau_syn=10.0), -1),                 # tau_m == tau_syn
    (dict(d_max_steps=101), -2),              # delay beyond the ring
    (dict(t_ref=30.0), -2),                   # t_ref / h > 255
    (dict(pop_size=[0, 1000]), -1),
    (dict(h=0.0), -1),
    (dict(w_mean=[[1e5, -351.2], [87.8, -351.2]]), -2),   # weight beyond int32 in 2^-16 pA
])
def test_invalid_configurations(change, code):
    w = workloads.balanced().replace(**change)
    with pytest.raises(mc.MCError) as e:
        mc.Network(w, host_only=True)
    assert e.value.code == code


def test_bernoulli_probability_range():
    w = workloads.microcircuit(scale=0.01)
    conn = [list(r) for r in w.conn]
    conn[0][0] = 1.5
    with pytest.raises(mc.MCError) as e:
        mc.Network(w.replace(conn=conn), host_only=True)
    assert e.value.code == -1


def test_host_only_handle_refuses_device_calls():
    net = mc.Network(workloads.balanced().replace(pop_size=[40, 10]), host_only=True)
    with pytest.raises(mc.MCError) as e:
        net.simulate(1)
    assert e.value.code == -5
    with pytest.raises(mc.MCError):
        net.state()


def test_null_arguments():
    L = mc.lib()
    h = C.c_void_p()
    assert L.mc_build_network(None, C.byref(h)) == -1
    assert L.mc_simulate(None, 1) == -5
    assert L.mc_strerror(-8) == b"recomputation did not reproduce the recorded spikes"


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU only and says so for --gpus N > 1."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_energy_meter_windows():
    """The package energy accumulator advances about once per second: power
    over a window is taken over the whole update intervals inside it, and a
    stray reading (timestamp out of order) or a repeat is ignored."""
    import bench
    m = bench.EnergyMeter.__new__(bench.EnergyMeter)
    m.samples = []
    s = 1_000_000_000
    # (host s, joules, counter ns): 300 W idle for 3 s, then 550 W
    for t, j, ts in [(0.0, 0.0, 10 * s), (0.5, 0.0, 10 * s), (1.0, 300.0, 11 * s), (1.4, 1e9, 3 * s),
                     (2.0, 600.0, 12 * s), (3.0, 900.0, 13 * s), (4.0, 1450.0, 14 * s), (5.0, 2000.0, 15 * s),
                     (6.0, 2550.0, 16 * s)]:
        m.add(t, j, ts)
    assert [x[0] for x in m.samples] == [0.0, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0]
    p, secs = m.power(-0.1, 3.0)
    assert p == 300.0 and secs == 3.0
    p, secs = m.power(3.2, 6.0)            # the interval (3, 4] starts before the window
    assert p == 550.0 and secs == 2.0
    assert m.power(3.2, 3.9) == (None, 0.0)
