"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Spike rasters, state bit patterns (y, I, r), the logical input ring and the
event counters must be identical: every input sum is an exact integer sum and
the FP64 update has a fixed operation order on both sides."""
import numpy as np
import pytest

import oracle
from paper_2111_04398_amd import mc, workloads
from test_oracle_builder import tiny_bernoulli, tiny_fixed
from test_oracle_dynamics import lone_neuron

pytestmark = pytest.mark.gpu


def assert_same(net, o, ring_depth=128, what=""):
    s, i = net.spikes()
    os_, oi = o.raster()
    assert len(s) == len(os_), (what, len(s), len(os_))
    assert np.array_equal(s, os_) and np.array_equal(i, oi), what
    y, I, r = net.state()
    oy, oI, orr = o.state()
    assert np.array_equal(y.view(np.uint64), oy.view(np.uint64)), what
    assert np.array_equal(I.view(np.uint64), oI.view(np.uint64)), what
    assert np.array_equal(r, orr), what
    if ring_depth:
        assert np.array_equal(net.ring(ring_depth), o.ring(ring_depth)), what
    c = net.counters()
    sp, ev = o.counters()
    assert c["events"] == ev and np.array_equal(c["spikes_per_pop"], sp), what
    assert c["step"] == o.step


def test_single_input_response():
    w = lone_neuron()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.inject(0, 0, 5754061)
    o.inject(0, 0, 5754061)
    for _ in range(5):
        net.simulate(40)
        o.run(40)
        assert_same(net, o, what="psp")


@pytest.mark.parametrize("ie", [300.0, 400.0, 1000.0])
def test_dc_drive(ie):
    w = lone_neuron(i_e=ie)
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.simulate(1500)
    o.run(1500)
    assert_same(net, o, what=f"dc {ie}")


@pytest.mark.parametrize("mk", [tiny_fixed, tiny_bernoulli])
def test_tiny_networks(mk):
    w = mk()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.simulate(2000)
    o.run(2000)
    assert len(o.raster()[0]) > 100
    assert_same(net, o, what=w.name)


def test_balanced_network_full_protocol():
    """The 5,000-neuron balanced network: 1000 presim steps then 10^4 steps
    (1 s of model time); compared after presim and at the end."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.simulate(w.presim_steps)
    o.run(w.presim_steps)
    assert_same(net, o, what="presim")
    net.simulate(w.sim_steps)
    o.run(w.sim_steps)
    assert_same(net, o, what="sim")
    assert o.counters()[1] > 10_000_000


@pytest.mark.parametrize("scheme,block,npw,spg", [
    (0, 64, 64, 1), (0, 256, 256, 1000), (0, 256, 1024, 7), (0, 1024, 512, 333), (0, 128, 16, 50), (0, 256, 256, 0),
    (1, 512, 0, 1000), (1, 256, 0, 100), (1, 512, 64, 7), (1, 512, 512, 250), (1, 512, 200, 0), (1, 128, 24, 50),
    (1, 64, 64, 50), (1, 512, 0, 1),
    (2, 256, 256, 1000), (2, 64, 16, 7), (2, 1024, 1024, 0), (2, 128, 100, 33),
    (3, 256, 0, 1000), (3, 256, 16, 7), (3, 512, 2048, 0), (3, 128, 100, 33), (3, 64, 384, 50), (3, 512, 0, 1),
    (3, 256, 4092, 20)])
def test_launch_configuration_invariance(scheme, block, npw, spg):
    """Every launch shape of every scheme gives identical bits (integer sums,
    fixed FP order).  (1, 64, 64) runs the persistent scheme with one
    wavefront per workgroup, which polls and then delivers by itself.
    Persistent neurons_per_wg = 512 leaves room for only ~30 delay steps in
    LDS, so most events take the far (global) path; the target-owner shapes
    range from 16 to 1024 targets per delivery block; the bucket scheme
    from 16 to 4092 targets per workgroup (1 to 4 quads per thread)."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.set_launch(scheme=scheme, block=block, neurons_per_wg=npw, steps_per_graph=spg)
    net.simulate(1200)
    o.run(1200)
    assert_same(net, o, what=f"{scheme},{block},{npw},{spg}")


@pytest.mark.parametrize("npw", [0, 512])
def test_persistent_launches_shorter_than_the_window(npw):
    """Direct persistent launches of 1 to 34 steps.  With the automatic block
    size the LDS delay window (101 steps) is longer than every launch, so the
    window the prologue takes from the ring and the one the epilogue writes
    back overlap; with 512 targets per workgroup it holds ~30 steps and most
    events take the far path through the ring's marked slots.  A 1-step launch
    publishes its only record before its ring scan.  Every call gives the
    oracle's bits and is timed as one launch by the call's own events."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.set_launch(scheme=1, block=512, neurons_per_wg=npw, steps_per_graph=0)
    dl = net.persist_shape()["lds_steps"]
    assert (dl > 34) if npw == 0 else (dl < 34), dl
    net.reserve(600)
    net.simulate(300)
    o.run(300)
    for k in (1, 2, 3, 1, 5, 8, 13, 1, 1, 21, 34, 2):
        net.simulate(k)
        o.run(k)
        t = net.last_kernel_ms()
        assert t["launches"] == 1 and t["steps"] == k and t["ms"] == net.last_simulate_ms(), (k, t)
        if k == 1:
            assert_same(net, o, what=f"after a 1-step launch at step {o.step}")
    assert_same(net, o, what="short launches")


@pytest.mark.parametrize("scheme,block,npw", [(1, 512, 0), (1, 512, 512), (3, 256, 0), (0, 256, 256)])
def test_injections_ahead_between_launches(scheme, block, npw):
    """Inputs injected 1 to d_max steps ahead (the oracle's ring holds d_max
    + 1 steps) between persistent launches of 1 to 120 steps.  With 512
    targets per workgroup the LDS window holds ~30 steps, so most reach the
    kernel through the ring's far slots, which the raised horizon makes the
    next launch's scan read and mark.  The trajectory stays the oracle's
    given the same injections; likewise for the bucket scheme and the step
    kernels."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.set_launch(scheme=scheme, block=block, neurons_per_wg=npw, steps_per_graph=0)
    net.reserve(1000)
    net.simulate(50)
    o.run(50)
    rng = np.random.default_rng(11 + npw)
    depth = w.to_dict()["d_max_steps"] + 1
    for steps in (1, 7, 40, 3, 90, 2, 120, 5):
        for _ in range(6):
            k, i = int(rng.integers(1, depth)), int(rng.integers(0, net.N))
            v = int(rng.integers(-6_000_000, 6_000_000))
            net.inject(k, i, v)
            o.inject(k, i, v)
        net.simulate(steps)
        o.run(steps)
    assert_same(net, o, what=f"injections ahead, launch {scheme},{block},{npw}")


# the launch shapes mc_tune times (same list and steps per graph)
TUNER_CANDIDATES = [(1, 512, 0, 10000, 0), (1, 256, 0, 10000, 0), (1, 512, 256, 10000, 0), (1, 512, 512, 10000, 0),
                    (1, 256, 128, 10000, 0), (0, 256, 256, 1000, 0), (0, 256, 256, 1000, 1), (0, 256, 1024, 1000, 0),
                    (0, 512, 512, 1000, 0), (0, 512, 512, 1000, 1), (0, 128, 128, 1000, 0), (0, 128, 128, 1000, 1),
                    (3, 192, 0, 10000, 0), (3, 256, 0, 10000, 0), (3, 512, 0, 10000, 0), (3, 128, 0, 10000, 0)]


def test_every_autotuner_candidate_gives_the_same_bits():
    """Whatever mc_tune picks, the trajectory is the oracle's: every
    candidate shape, run from the same state, gives identical bits."""
    w = workloads.balanced()
    o = oracle.Oracle(w.to_dict())
    o.run(900)
    for c in TUNER_CANDIDATES:
        net = mc.Network(w)
        net.set_launch(scheme=c[0], block=c[1], neurons_per_wg=c[2], steps_per_graph=c[3], rows_per_wave=c[4])
        net.simulate(900)
        assert_same(net, o, ring_depth=128, what=f"candidate {c}")
        net.close()


@pytest.mark.parametrize("block", [512, 256])
def test_producer_order_listing_after_early_near_delivery(block, monkeypatch):
    """The persistent scheme adds the near events of the first listed ids
    while the poll goes on; a step that is then listed in producer order
    after the wait takes those events out again before delivering the step.
    With the listing threshold lowered to 8 spikes (a test hook, honoured by
    the phase-timing kernel that mc_profile_phases runs), most steps of the
    balanced network (~15 spikes each) take that path, with the early
    delivery in a wavefront without targets: the trajectory is still the
    oracle's, bit for bit."""
    monkeypatch.setenv("MC_PERSIST_LIST_CAP", "8")
    w = workloads.balanced()
    o = oracle.Oracle(w.to_dict())
    o.run(900)
    net = mc.Network(w)
    net.set_launch(scheme=1, block=block, neurons_per_wg=0, steps_per_graph=300)
    net.profile_phases(900)
    assert_same(net, o, ring_depth=128, what=f"list threshold 8, block {block}")
    net.close()


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_all_delays_one_step(scheme):
    """Every synapse with the smallest delay (one step): every event must be
    in place by the next update, so a missing wait anywhere in the exchange
    would show.  In the persistent scheme every event takes the near path."""
    w = workloads.balanced().replace(name="delay1", d_max_steps=1)
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    assert set(np.unique(net.synapses()[3])) == {1}
    net.set_launch(scheme=scheme, block=512 if scheme == 1 else 256, neurons_per_wg=0 if scheme in (1, 3) else 256,
                   steps_per_graph=100)
    net.simulate(1000)
    o.run(1000)
    assert o.counters()[1] > 1_000_000
    assert_same(net, o, what=f"delay1 {scheme}")


@pytest.mark.parametrize("scheme,block,npw,spg", [(0, 256, 256, 100), (1, 512, 0, 100), (1, 256, 64, 7),
                                                   (2, 256, 256, 100), (3, 256, 0, 100), (3, 512, 2048, 100),
                                                   (3, 64, 64, 7)])
def test_synchronous_bursts(scheme, block, npw, spg):
    """A DC current far above threshold makes every neuron fire at its first
    free step: all 5,000 fire together every 21 steps.  That is the densest
    raster the refractory period allows (the raster bound is met exactly) and,
    in the persistent schemes, more spikes in one step than their LDS spike
    lists hold (the branches that deliver such a step at once, or in chunks
    read back from the records).  With 2048 targets per workgroup a burst
    brings ~1e6 events to one workgroup, far more than its buckets hold: the
    overflow goes to the ring."""
    w = workloads.balanced().replace(name="bursts", i_e=1.0e5)
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.set_launch(scheme=scheme, block=block, neurons_per_wg=npw, steps_per_graph=spg)
    net.simulate(300)
    o.run(300)
    s, _ = o.raster()
    assert len(s) == 5000 * len(range(0, 300, 21)) and set(np.unique(s)) == set(range(0, 300, 21))
    assert_same(net, o, what=f"bursts {scheme},{block},{npw},{spg}")


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_silent_network(scheme):
    """No drive and no current: no neuron ever fires, nothing is delivered,
    and the membrane decays by the same propagator bits on both sides."""
    w = workloads.balanced().replace(name="silent", nu_ext=0.0, v0_lo=-65.0, v0_hi=-50.5)
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.set_launch(scheme=scheme, block=512 if scheme == 1 else 256, neurons_per_wg=0 if scheme in (1, 3) else 256,
                   steps_per_graph=50)
    net.simulate(400)
    o.run(400)
    assert len(o.raster()[0]) == 0 and o.counters()[1] == 0
    assert_same(net, o, what=f"silent {scheme}")


def test_persistent_scheme_at_its_largest_shape():
    """131,072 neurons in 512 workgroups of 256 targets: the most workgroups
    the persistent scheme runs (two per compute unit, each polling 512
    records), leaving 7 steps of input in LDS, so most events take the far
    path.  A shape that cannot be co-resident is refused before any launch."""
    w = workloads.balanced().replace(name="max_persistent", pop_size=[104856, 26216],
                                     conn=[[40.0, 10.0], [40.0, 10.0]])
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    assert net.N == 131072
    with pytest.raises(mc.MCError) as e:     # 512 workgroups of 512 threads: two per CU do not fit the registers
        net.set_launch(scheme=1, block=512, neurons_per_wg=256, steps_per_graph=100)
    assert e.value.code == -2 and "co-resident" in str(e.value)
    net.set_launch(scheme=1, block=256, neurons_per_wg=256, steps_per_graph=100)
    assert net.persist_shape()["workgroups"] == 512 and net.persist_shape()["targets_per_wg"] == 256
    net.simulate(300)
    o.run(300)
    assert len(o.raster()[0]) > 1000
    assert_same(net, o, ring_depth=16, what="max persistent")


@pytest.mark.parametrize("name", ["tiny_fixed", "tiny_bernoulli", "adjoint_small", "batched_4", "balanced",
                                  "microcircuit"])
def test_device_connection_drawing_builds_the_oracles_network(name):
    """MC_FLAG_DEVICE_CONNECT draws the connections on the device (the pair
    tests of the Bernoulli rule, the source draws of the fixed in-degree
    rule); the synapse store (rows, targets, weights, delays) equals the
    oracle's bit for bit, instance by instance for the batch, and so does
    the trajectory."""
    w = {"tiny_fixed": tiny_fixed, "tiny_bernoulli": tiny_bernoulli, "adjoint_small": workloads.adjoint_small,
         "batched_4": lambda: workloads.batched(n_instances=4, sim_steps=300),
         "balanced": workloads.balanced, "microcircuit": workloads.microcircuit}[name]()
    net = mc.Network(w, device_connect=True)
    rp, tg, wq, d = net.synapses()
    off = net.instance_offsets()
    for b in range(net.n_instances):
        o = oracle.Oracle(w.instance(b).to_dict())
        orp, otg, owq, od = o.synapses()
        m0, m1 = rp[off[b]], rp[off[b + 1]]
        assert np.array_equal(rp[off[b]:off[b + 1] + 1] - m0, orp), (name, b)
        assert np.array_equal(tg[m0:m1] - off[b], otg), (name, b)
        assert np.array_equal(wq[m0:m1], owq) and np.array_equal(d[m0:m1], od), (name, b)
        del o, orp, otg, owq, od
    del rp, tg, wq, d
    if net.n_instances == 1 and net.M < 10_000_000:
        o = oracle.Oracle(w.to_dict())
        net.set_launch(scheme=0, block=256, neurons_per_wg=256, steps_per_graph=100)
        net.simulate(200)
        o.run(200)
        assert_same(net, o, what=name)


def test_recording_allocation_failure_keeps_the_handle_usable():
    """A raster reservation beyond device memory (2e6 steps of the 64-instance
    batch: ~570 GB at the worst-case spike bound) returns MC_ERR_OOM and
    leaves the previous capacity in place: the network then simulates exactly
    as an untouched twin does."""
    w = workloads.batched(sim_steps=300)
    net = mc.Network(w, device_connect=True)
    twin = mc.Network(w, device_connect=True)
    with pytest.raises(mc.MCError) as e:
        net.reserve(2_000_000)
    assert e.value.code == -3 and "capacity left" in str(e.value)
    for x in (net, twin):
        x.simulate(300)
    s0, i0 = net.spikes()
    s1, i1 = twin.spikes()
    assert len(s0) > 0 and np.array_equal(s0, s1) and np.array_equal(i0, i1)
    assert net.counters()["events"] == twin.counters()["events"]


def test_device_connection_drawing_refuses_host_only():
    with pytest.raises(mc.MCError) as e:
        mc.Network(tiny_bernoulli(), host_only=True, device_connect=True)
    assert e.value.code == mc.MC_ERR_INVALID_ARG


@pytest.mark.parametrize("mk", [tiny_fixed, tiny_bernoulli])
def test_tiny_networks_persistent(mk):
    w = mk()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.set_launch(scheme=1, block=256, neurons_per_wg=0, steps_per_graph=500)
    net.simulate(2000)
    o.run(2000)
    assert_same(net, o, what=w.name)


def test_scheme_switch_midway():
    """Switching between the schemes in the middle of a run changes nothing."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    order = [1, 0, 3, 2, 1, 3, 3, 1, 2, 0, 2]
    for k, sch in enumerate(order):
        net.set_launch(scheme=sch, block=512 if sch == 1 else 256, neurons_per_wg=0 if sch in (1, 3) else 256,
                       steps_per_graph=97 + k)
        net.simulate(311)
    o.run(len(order) * 311)
    assert_same(net, o, what="switch")


def test_resume_and_checkpoint():
    """simulate(a) + simulate(b) == simulate(a+b); save, continue, load, rerun
    reproduces the same trajectory; a launch change in between changes nothing."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.simulate(300)
    net.simulate(77)
    blob = net.save_state()
    net.set_launch(block=512, neurons_per_wg=128, steps_per_graph=64)
    net.simulate(500)
    o.run(877)
    assert_same(net, o, what="continue")
    s_first, i_first = net.spikes(377, 877)
    net.load_state(blob)
    assert net.counters()["step"] == 377
    net.simulate(500)
    assert_same(net, o, what="reload")
    s2, i2 = net.spikes(377, 877)
    assert np.array_equal(s_first, s2) and np.array_equal(i_first, i2)


@pytest.mark.parametrize("scheme", [1, 3])
def test_short_rewinds_onto_other_states(scheme):
    """Loading a state a few steps back, alternately the network's own and
    that of another seed (same shape), then simulating: every run matches
    the oracle started from that state.  In the persistent scheme the spike
    records of the abandoned steps carry the same step tags as the steps
    simulated again; they are cleared before every launch."""
    wa, wb = workloads.balanced(seed=1), workloads.balanced(seed=2)
    a, b = mc.Network(wa), mc.Network(wb)
    for net in (a, b):
        net.set_launch(scheme=scheme, block=512, neurons_per_wg=0, steps_per_graph=1000)
        net.simulate(100)
    blob_a, blob_b = a.save_state(), b.save_state()
    # expected: seed-1 network continued from its own state and from seed 2's
    own = oracle.Oracle(wa.to_dict())
    own.run(100)
    other = oracle.Oracle(wa.to_dict())
    other.run(100)
    other.set_state(*b.state())
    diff = b.ring() - other.ring()
    for k, i in zip(*np.nonzero(diff)):
        other.inject(int(k), int(i), int(diff[k, i]))
    assert np.array_equal(other.ring(), b.ring())
    runs = 4
    own.run(runs)
    other.run(runs)
    expect = {}
    for name, o in (("own", own), ("other", other)):
        s, i = o.raster()
        keep = s >= 100
        expect[name] = (s[keep], i[keep])
    for rep in range(8):
        name = ("other", "own")[rep % 2]
        a.load_state(blob_b if name == "other" else blob_a)
        a.simulate(1 + rep % runs)
        s, i = a.spikes(100, 200)
        es, ei = expect[name]
        m = es < 100 + 1 + rep % runs
        assert np.array_equal(s, es[m]) and np.array_equal(i, ei[m]), (rep, name)


@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_batched_instances_match_standalone(scheme):
    """Instances of a batch are bit-identical to their standalone runs, in
    every scheme (target-owner blocks of 64 targets: several per instance,
    none spanning two instances)."""
    base = workloads.microcircuit()
    scales = [0.01, 0.013, 0.0071, 0.02]
    w = base.replace(inst_scale=scales, inst_seed=[1001, 1002, 1003, 1004])
    net = mc.Network(w)
    if scheme == 1:
        net.set_launch(scheme=1, block=512, neurons_per_wg=0, steps_per_graph=500)
    elif scheme == 2:
        net.set_launch(scheme=2, block=256, neurons_per_wg=64, steps_per_graph=300)
    elif scheme == 3:
        net.set_launch(scheme=3, block=64, neurons_per_wg=96, steps_per_graph=300)
    net.simulate(1500)
    s, i = net.spikes()
    y, I, r = net.state()
    off = net.instance_offsets()
    total_events = 0
    for b in range(len(scales)):
        o = oracle.Oracle(w.instance(b).to_dict())
        o.run(1500)
        os_, oi = o.raster()
        m = (i >= off[b]) & (i < off[b + 1])
        assert np.array_equal(s[m], os_) and np.array_equal(i[m] - off[b], oi)
        oy, oI, orr = o.state()
        assert np.array_equal(y[off[b]:off[b + 1]].view(np.uint64), oy.view(np.uint64))
        assert np.array_equal(r[off[b]:off[b + 1]], orr)
        total_events += o.counters()[1]
    assert net.counters()["events"] == total_events


@pytest.mark.slow
def test_batched_c2_full_shape_matches_per_instance_oracles():
    """The 64-instance batch at its benchmark shape (seeds 1001-1064, scales
    0.05-0.25, 750,775 neurons, ~5e8 synapses) under the launch the
    autotuner picks for it, 1000 presim steps and 300 more: every
    instance's raster, y/I/r bits, first 8 logical ring slots and event and
    spike counters equal its standalone oracle's, run one instance after
    another on the host."""
    w = workloads.batched()
    runs = []
    for how in ("tuned", "buckets"):
        net = mc.Network(w, device_connect=True)
        assert net.n_instances == 64 and net.N == 750_775
        net.simulate(100)
        if how == "tuned":
            launch = net.tune(200)
        else:
            net.set_launch(scheme=3, block=256, neurons_per_wg=0, steps_per_graph=1000)
            launch = net.get_launch()
        print(f"c2 {how} launch: {launch} shape {net.persist_shape()}", flush=True)
        net.simulate(w.presim_steps - 100)
        net.simulate(300)
        runs.append((how, net.spikes(), net.state(), net.ring(8), net.counters()))
        off = net.instance_offsets()
        net.close()
    ev_total, sp_total = 0, np.zeros(w.n_pops, np.int64)
    for b in range(64):
        o = oracle.Oracle(w.instance(b).to_dict())
        o.run(w.presim_steps + 300)
        os_, oi = o.raster()
        oy, oI, orr = o.state()
        oring = o.ring(8)
        sl = slice(off[b], off[b + 1])
        for how, (s, i), (y, I, r), ring, _ in runs:
            m = (i >= off[b]) & (i < off[b + 1])
            assert np.array_equal(s[m], os_) and np.array_equal(i[m] - off[b], oi), (b, how)
            assert np.array_equal(y[sl].view(np.uint64), oy.view(np.uint64)), (b, how)
            assert np.array_equal(I[sl].view(np.uint64), oI.view(np.uint64)), (b, how)
            assert np.array_equal(r[sl], orr), (b, how)
            assert np.array_equal(ring[:, sl], oring), (b, how)
        sp, ev = o.counters()
        ev_total += ev
        sp_total += sp
        del o
        print(f"c2 instance {b}: {len(os_)} spikes equal in both launches", flush=True)
    for how, (s, i), _, _, c in runs:
        assert c["events"] == ev_total and np.array_equal(c["spikes_per_pop"], sp_total), how
        assert c["step"] == w.presim_steps + 300 and len(s) > 100_000


@pytest.fixture(scope="module")
def micro_oracle_runs():
    """Oracle trajectory of the full microcircuit: after 1000 and 1300 steps."""
    w = workloads.microcircuit()
    o = oracle.Oracle(w.to_dict())
    o.run(1000)
    a = (o.raster(), o.state(), o.ring(8), o.counters())
    o.run(300)
    b = (o.raster(), o.state(), o.ring(8), o.counters())
    return w, o.N, o.M, a, b


@pytest.mark.slow
@pytest.mark.parametrize("scheme", [0, 1, 2, 3])
def test_full_microcircuit_parity(micro_oracle_runs, scheme):
    """The full-scale microcircuit (77,169 neurons, ~3e8 synapses): raster,
    state bits and the first logical ring slots equal to the oracle's after
    the 1000-step presim and after 300 further steps, in both schemes (the
    benchmark's launch configuration is the default of the scheme)."""
    w, N, M, a, b = micro_oracle_runs
    net = mc.Network(w)
    if scheme == 1:
        net.set_launch(scheme=1, block=512, neurons_per_wg=0, steps_per_graph=1000)
    elif scheme == 2:
        net.set_launch(scheme=2, block=256, neurons_per_wg=256, steps_per_graph=1000)
    elif scheme == 3:
        net.set_launch(scheme=3, block=256, neurons_per_wg=0, steps_per_graph=1000)
    assert (net.N, net.M) == (N, M)
    for steps, (ras, st, ring, cnt) in ((1000, a), (300, b)):
        net.simulate(steps)
        s, i = net.spikes()
        assert np.array_equal(s, ras[0]) and np.array_equal(i, ras[1])
        y, I, r = net.state()
        assert np.array_equal(y.view(np.uint64), st[0].view(np.uint64))
        assert np.array_equal(I.view(np.uint64), st[1].view(np.uint64))
        assert np.array_equal(r, st[2])
        assert np.array_equal(net.ring(8), ring)
        c = net.counters()
        assert c["events"] == cnt[1] and np.array_equal(c["spikes_per_pop"], cnt[0])
    assert len(b[0][0]) > 50_000


def test_delivery_replay_matches_independent_sum():
    """The one-launch replay of the recorded spikes of steps [100, 400) puts
    into slot k exactly the sum of w over all synapses (i -> j, d) of spikes
    (t, i) with t - 100 + d = k -- recomputed here with numpy from the
    oracle's store and raster."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.set_launch(scheme=1, block=512, neurons_per_wg=0, steps_per_graph=1000)
    net.simulate(450)
    o.run(450)
    ms, ev, ring = net.replay_delivery(100, 400, want_ring=True)
    rp, tg, wq, d = o.synapses()
    s, i = o.raster()
    sel = (s >= 100) & (s < 400)
    expect = np.zeros_like(ring)
    events = 0
    for t, src in zip(s[sel], i[sel]):
        lo, hi = rp[src], rp[src + 1]
        np.add.at(expect, (t - 100 + d[lo:hi].astype(np.int64), tg[lo:hi]), wq[lo:hi].astype(np.int64))
        events += hi - lo
    assert ev == events > 0
    assert np.array_equal(ring, expect)
    assert ms > 0


def test_autotuner_and_phase_profile_keep_the_trajectory():
    """mc_tune times candidate launches on copies of the state and restores
    it; mc_profile_phases simulates exactly as mc_simulate does.  Both leave
    the trajectory bit-identical to the oracle's."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.simulate(300)
    best = net.tune(150)
    assert net.counters()["step"] == 300
    net.simulate(400)
    net.set_launch(scheme=1, block=512, neurons_per_wg=0, steps_per_graph=100)
    ph = net.profile_phases(300)
    assert ph["total"] > 0 and net.phase_table().shape == (net.persist_shape()["workgroups"], 8)
    net.simulate(200)
    net.set_launch(scheme=3, block=256, neurons_per_wg=0, steps_per_graph=100)
    ph = net.profile_phases(200)
    assert ph["total"] > 0 and ph["deliver"] > 0
    assert net.phase_table().shape == (net.persist_shape()["workgroups"], 8)
    net.simulate(100)
    o.run(1500)
    assert_same(net, o, what=f"tuned {best}")


def test_network_lives_in_torch_allocator_memory():
    """With the allocator hooks of mc_config every device buffer of the
    network (synapse store, state, ring, raster, the persistent scheme's
    tables) comes from torch's caching allocator and goes back to it; the
    trajectory is the oracle's."""
    import torch
    live, total = {}, {"allocs": 0, "frees": 0, "bytes": 0}

    def fa(nbytes):
        p = torch.cuda.caching_allocator_alloc(nbytes)
        assert p not in live                         # torch may hand out a freed block again
        live[p] = nbytes
        total["allocs"] += 1
        total["bytes"] += nbytes
        return p

    def ff(ptr):
        assert ptr in live
        del live[ptr]
        torch.cuda.caching_allocator_delete(ptr)
        total["frees"] += 1

    w = workloads.balanced()
    net = mc.Network(w, allocator=(fa, ff))
    o = oracle.Oracle(w.to_dict())
    assert total["bytes"] >= 9 * net.M               # the synapse store came from torch
    net.set_launch(scheme=1, block=512, neurons_per_wg=0, steps_per_graph=200)
    net.simulate(500)
    o.run(500)
    assert_same(net, o, what="torch allocator")
    net.close()
    assert not live and total["frees"] == total["allocs"] > 10


@pytest.mark.parametrize("block,npw,spg", [(256, 256, 1000), (64, 64, 1), (1024, 512, 333)])
def test_rows_per_wavefront_delivery(block, npw, spg):
    """The step kernels' delivery with each wavefront walking whole rows
    gives the oracle's bits."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.set_launch(scheme=0, block=block, neurons_per_wg=npw, steps_per_graph=spg, rows_per_wave=1)
    net.simulate(800)
    o.run(800)
    assert_same(net, o, what=f"rows per wave {block},{npw},{spg}")


def test_tune_cache_skips_the_second_tuning(tmp_path, monkeypatch):
    """With MC_TUNE_CACHE set, the first mc_tune times the candidates and
    stores its choice under the network's shape and device; a second network
    of the same shape gets the stored launch without any timing (the cache
    file gains no line), and its trajectory is the oracle's."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("MC_TUNE_CACHE", str(cache))
    w = workloads.balanced()
    a = mc.Network(w)
    first = a.tune(100)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split()[1:6] == [str(first[k]) for k in
                                                         ("scheme", "block", "neurons_per_wg", "steps_per_graph",
                                                          "rows_per_wave")]
    b = mc.Network(w.replace(seed=9))
    second = b.tune(100)
    assert second == first and cache.read_text().splitlines() == lines
    o = oracle.Oracle(w.replace(seed=9).to_dict())
    b.simulate(500)
    o.run(500)
    assert_same(b, o, what="cached launch")


def test_probes_and_launch_timing_leave_the_trajectory():
    """The memory probes (streaming read, slot-major atomics, the empty
    persistent exchange) measure within physical bounds and leave the
    network untouched; the persistent kernel's launches are timed one by
    one (graph replays and the direct remainder) and their summed time lies
    inside the simulate span; a call that is one launch is timed by the
    call's span.  The trajectory stays the oracle's."""
    w = workloads.balanced()
    net, o = mc.Network(w), oracle.Oracle(w.to_dict())
    net.simulate(100)
    with pytest.raises(mc.MCError) as e:               # the exchange probe needs a persistent scheme
        net.probe_exchange(100)
    assert e.value.code == mc.MC_ERR_STATE
    assert net.last_kernel_ms()["launches"] == 0        # step kernels: no persistent launch
    gbs = net.probe_stream(256 << 20)
    assert 500.0 < gbs < 8500.0, gbs
    for pattern in (0, 1):
        rate = net.probe_atomics(128, pattern)
        assert 1.0 < rate < 1000.0, rate                # 1e9 adds/s
    for scheme, block in ((1, 512), (3, 256)):
        net.set_launch(scheme=scheme, block=block, neurons_per_wg=0, steps_per_graph=100)
        floor = net.probe_exchange(500) if scheme == 1 else None   # the LDS-window scheme's shape only
        net.reserve(300)
        net.simulate(250)                               # two graph replays of 100 steps, one direct launch of 50
        k = net.last_kernel_ms()
        assert k["launches"] == 3 and k["steps"] == 250
        assert 0.0 < k["ms"] <= net.last_simulate_ms()
        if floor is not None:
            assert 0.0 < floor * 250 * 1e-3 <= k["ms"] * 1.5, (floor, k)
        net.simulate(50)                                # one direct launch: timed by the call's own events
        k = net.last_kernel_ms()
        assert k["launches"] == 1 and k["steps"] == 50 and k["ms"] == net.last_simulate_ms()
    o.run(700)
    assert_same(net, o, what="after probes and timed launches")
