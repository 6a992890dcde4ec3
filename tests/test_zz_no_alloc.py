"""The allocation-free entry point (mc_simulate_noalloc) against mc_simulate,
through the C interface: the same raster, state bits, logical ring and
counters, on two calls in a row (the second on a smaller network, so the
scratch shared by every call on the GPU is reused with a smaller shape),
and both equal to the oracle.  Also: the refusals that keep it allocation-
free (another scheme, too little raster room)."""
import numpy as np
import pytest

import oracle
from paper_2111_04398_amd import mc, workloads
from test_gpu_parity import assert_same
from test_oracle_builder import tiny_bernoulli

pytestmark = pytest.mark.gpu


def run_pair(w, steps, block, npw):
    ref, nal = mc.Network(w), mc.Network(w)
    for net in (ref, nal):
        net.set_launch(scheme=1, block=block, neurons_per_wg=npw, steps_per_graph=1000)
        net.reserve(steps)
    ref.simulate(steps)
    nal.simulate_noalloc(steps)
    o = oracle.Oracle(w.to_dict())
    o.run(steps)
    assert_same(ref, o, what=f"simulate {w.name}")
    assert_same(nal, o, what=f"noalloc {w.name}")
    assert nal.last_kernel_ms()["launches"] == 1
    return ref, nal


def test_noalloc_matches_simulate_on_two_calls():
    big, _ = run_pair(workloads.balanced(), 600, 512, 0)           # 40 workgroups of 128 targets
    assert big.persist_shape()["workgroups"] > 8
    small, nal = run_pair(tiny_bernoulli(), 400, 256, 0)            # fewer workgroups: the same scratch, smaller
    assert small.persist_shape()["workgroups"] < big.persist_shape()["workgroups"]
    # continuing with both entry points alternately stays on the trajectory
    nal.reserve(300)
    nal.simulate(150)
    nal.simulate_noalloc(150)
    o = oracle.Oracle(tiny_bernoulli().to_dict())
    o.run(700)
    assert_same(nal, o, what="alternating")


def test_noalloc_refusals():
    w = workloads.balanced()
    net = mc.Network(w)
    with pytest.raises(mc.MCError) as e:          # step kernels: no persistent scratch to take
        net.simulate_noalloc(10)
    assert e.value.code == -5
    net.set_launch(scheme=1, block=512, neurons_per_wg=0, steps_per_graph=1000)
    with pytest.raises(mc.MCError) as e:          # more steps than the raster holds without a drain
        net.simulate_noalloc(10_000_000)
    assert e.value.code == mc.MC_ERR_BUFFER_TOO_SMALL
    net.simulate_noalloc(0)
    assert net.counters()["step"] == 0
