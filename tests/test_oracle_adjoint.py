"""Pins of the oracle's reverse-time adjoint: against 50-digit central
differences recomputed here from the recorded trajectory, and against the
oracle's own quad-precision finite differences on a scale-0.1 microcircuit."""
import mpmath
import numpy as np
import pytest

import oracle
from paper_2111_04398_amd import workloads

Y_STAR = -58.0 - (-65.0)


def tiny_adjoint_net(seed=11):
    w = workloads.balanced(seed=seed)
    return w.replace(pop_size=[4, 2], conn=[[2.0, 1.0], [2.0, 1.0]], k_ext=[2400.0, 2400.0])


def mp_loss_of_neuron(types, x_int, y0, hits, delta, P, S, I0=0.0):
    """sum_n (y_{n+1} - y*)^2 for one neuron with frozen step types, input
    x_n = x_int 2^-16 + delta at the listed steps, from (y0, I0); 50-digit
    arithmetic with the FP64 propagator values."""
    P11, P21, P22 = (mpmath.mpf(float(v)) for v in P[:3])
    y, I, L = mpmath.mpf(float(y0)), mpmath.mpf(float(I0)), mpmath.mpf(0)
    ys = mpmath.mpf(Y_STAR)
    for n in range(S):
        x = mpmath.mpf(int(x_int[n])) / 65536
        if hits[n]:
            x += delta
        t = types[n]
        if t == 0:
            y = P22 * y + P21 * I
        elif t == 1:
            y = mpmath.mpf(0)
        I = P11 * I + x
        L += (y - ys) ** 2
    return L


def test_adjoint_matches_50_digit_central_differences():
    """dL/dw for every synapse of a 6-neuron, 400-step network: the frozen-spike
    loss is quadratic in each weight, so the central difference with eps = 1e-3
    pA at 50 digits is the derivative; oracle FP64 adjoint within 1e-12."""
    mpmath.mp.dps = 50
    S = 400
    w = tiny_adjoint_net().to_dict()
    o = oracle.Oracle(w)
    N = o.N
    rp, tg, wq, d = o.synapses()
    loss, g = o.adjoint(S, Y_STAR)
    rs, ri = o.raster()
    assert 20 < len(rs) < 400
    P = o.propagators()
    P = (P[0], P[1], P[2])
    traces = []
    for j in range(N):
        oj = oracle.Oracle(w)
        traces.append(oj.trace(S, j))
    # loss recomputed from the traces
    L = mpmath.mpf(0)
    for j in range(N):
        L += mp_loss_of_neuron(traces[j][0], traces[j][1], traces[j][2][0], np.zeros(S, bool), 0, P, S)
    assert abs(loss - float(L / (N * S))) <= 1e-14 * abs(loss)
    src = np.repeat(np.arange(N), np.diff(rp))
    eps = mpmath.mpf("1e-3")
    n_nonzero = 0
    for k in range(len(tg)):
        i, j = int(src[k]), int(tg[k])
        hits = np.zeros(S, bool)
        for t in rs[ri == i]:
            if t + d[k] <= S - 1:
                hits[t + d[k]] = True
        types, x_int, ytr = traces[j]
        lp = mp_loss_of_neuron(types, x_int, ytr[0], hits, eps, P, S)
        lm = mp_loss_of_neuron(types, x_int, ytr[0], hits, -eps, P, S)
        fd = float((lp - lm) / (2 * eps) / (N * S))
        if not hits.any():
            assert g[k] == 0.0
            continue
        n_nonzero += 1
        assert abs(g[k] - fd) <= 1e-12 * abs(fd) + 1e-300, (k, g[k], fd)
    assert n_nonzero > 5
    mpmath.mp.dps = 40


def test_adjoint_from_a_later_step_matches_50_digit_central_differences():
    """A 60-step window that starts after 150 steps: the state there, with
    the input still pending from earlier spikes, is the initial condition, so
    only the window's own spikes carry weights the gradient sees (three
    synapses here have arrivals inside the window from earlier spikes only:
    their gradient is 0).  Every synapse against the 50-digit central
    difference, as from fresh."""
    mpmath.mp.dps = 50
    n0, S = 150, 60
    w = tiny_adjoint_net().to_dict()
    o = oracle.Oracle(w)
    o.run(n0)
    y0, I0, _ = o.state()
    pending = o.ring()
    before = len(o.raster()[0])
    N = o.N
    rp, tg, wq, d = o.synapses()
    loss, g = o.adjoint(S, Y_STAR)
    assert o.step == n0 + S
    rs, ri = o.raster()
    pre_s, pre_i = rs[:before], ri[:before]
    rs, ri = rs[before:], ri[before:]
    assert before > 3 and np.count_nonzero(pending) > 0 and len(rs) >= 3
    P = o.propagators()
    P = (P[0], P[1], P[2])
    traces = []
    for j in range(N):
        oj = oracle.Oracle(w)
        oj.run(n0)
        traces.append(oj.trace(S, j))
        assert traces[j][2][0] == y0[j]
    L = mpmath.mpf(0)
    for j in range(N):
        L += mp_loss_of_neuron(traces[j][0], traces[j][1], y0[j], np.zeros(S, bool), 0, P, S, I0[j])
    assert abs(loss - float(L / (N * S))) <= 1e-14 * abs(loss)
    src = np.repeat(np.arange(N), np.diff(rp))
    eps = mpmath.mpf("1e-3")
    n_nonzero = n_pre_only = 0
    for k in range(len(tg)):
        i, j = int(src[k]), int(tg[k])
        hits = np.zeros(S, bool)
        for t in rs[ri == i]:
            if t - n0 + d[k] <= S - 1:
                hits[t - n0 + d[k]] = True
        if not hits.any():
            assert g[k] == 0.0
            arr = pre_s[pre_i == i] + d[k]
            n_pre_only += int(np.any((arr >= n0) & (arr <= n0 + S - 1)))
            continue
        types, x_int, _ = traces[j]
        lp = mp_loss_of_neuron(types, x_int, y0[j], hits, eps, P, S, I0[j])
        lm = mp_loss_of_neuron(types, x_int, y0[j], hits, -eps, P, S, I0[j])
        fd = float((lp - lm) / (2 * eps) / (N * S))
        n_nonzero += 1
        assert abs(g[k] - fd) <= 1e-12 * abs(fd) + 1e-300, (k, g[k], fd)
    assert n_nonzero > 5 and n_pre_only > 0   # arrivals of pre-window spikes only: gradient 0
    mpmath.mp.dps = 40


@pytest.mark.slow
def test_adjoint_matches_quad_fd_on_scaled_microcircuit():
    """Scale 0.1 of the microcircuit, 2000 steps, 200 synapses with at least one
    in-window arrival: FP64 adjoint vs quad-precision central differences
    (eps = 1e-3 pA) within 1e-9 relative; synapses without arrivals have a
    gradient of exactly 0."""
    w = workloads.adjoint_small().to_dict()
    S = 2000
    o = oracle.Oracle(w)
    loss, g = o.adjoint(S, Y_STAR)
    rp, tg, wq, d = o.synapses()
    rs, ri = o.raster()
    # arrival test per synapse: a spike of its source with t + d <= S - 1
    first_spike = np.full(o.N, S, np.int64)
    np.minimum.at(first_spike, ri, rs)
    src = np.repeat(np.arange(o.N), np.diff(rp))
    has_arrival = first_spike[src] + d <= S - 1
    rng = np.random.default_rng(2024)
    sel = rng.choice(np.flatnonzero(has_arrival), 200, replace=False)
    fd = oracle.Oracle(w).fd(S, Y_STAR, 1e-3, sel)
    rel = np.abs(g[sel] - fd) / np.abs(fd)
    assert rel.max() <= 1e-9, rel.max()
    zero = np.flatnonzero(~has_arrival)
    assert zero.size > 0 and np.all(g[zero] == 0.0)
