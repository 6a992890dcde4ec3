"""Pins of the oracle's gradient step on the stored weights (w <- w - eta g,
stored again in units of 2^-16 pA, nearest with ties to even) and of its
reset to the initial state.

The expected stores are computed here in exact rational arithmetic
(``fractions.Fraction`` and Python's round-half-even ``round``) or from
closed forms, never with the oracle's floating-point expression."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from test_oracle_adjoint import Y_STAR, tiny_adjoint_net
from test_oracle_builder import tiny_fixed


@pytest.fixture()
def net():
    return oracle.Oracle(tiny_fixed().to_dict())


def stored(o):
    return o.synapses()[2].astype(np.int64)


def test_zero_rate_changes_nothing(net):
    w0 = stored(net)
    assert net.apply_gradient(np.random.default_rng(1).normal(size=net.M), 0.0)
    assert np.array_equal(stored(net), w0)


def test_gradient_equal_to_the_weights(net):
    """g = w (pA): eta = 1 zeroes every weight, eta = -1 doubles it, eta = 1/2
    halves it with ties to even (odd stored integers land on a half)."""
    w0 = stored(net)
    g = w0.astype(np.float64) / 65536.0
    a = oracle.Oracle(tiny_fixed().to_dict())
    assert a.apply_gradient(g, 1.0) and np.array_equal(stored(a), np.zeros_like(w0))
    b = oracle.Oracle(tiny_fixed().to_dict())
    assert b.apply_gradient(g, -1.0) and np.array_equal(stored(b), 2 * w0)
    c = oracle.Oracle(tiny_fixed().to_dict())
    assert c.apply_gradient(g, 0.5)
    expect = np.array([round(Fraction(int(v), 2)) for v in w0], np.int64)
    assert np.any(w0 % 2 == 1) and np.array_equal(stored(c), expect)


def test_integer_steps_and_rounding_of_fractions(net):
    """g = k 2^-16 pA for integers k and integer eta shift each stored weight
    by exactly -eta k; a general g and eta round w - eta g (exact rational)
    to the nearest integer multiple of 2^-16 pA, ties to even, in float64 and
    float32 gradients alike."""
    rng = np.random.default_rng(7)
    w0 = stored(net)
    k = rng.integers(-1000, 1000, size=net.M)
    assert net.apply_gradient(k.astype(np.float64) / 65536.0, 3.0)
    assert np.array_equal(stored(net), w0 - 3 * k)
    for dtype in (np.float64, np.float32):
        o = oracle.Oracle(tiny_fixed().to_dict())
        g = rng.normal(scale=5.0, size=o.M).astype(dtype)
        eta = 0.37
        assert o.apply_gradient(g, eta)
        # fl(eta g) is one rounding; the difference with w is formed exactly
        # here and then rounded once more, as the double subtraction does
        got = stored(o)
        for j in range(o.M):
            prod = Fraction(float(eta * float(g[j])))
            exact = Fraction(int(w0[j]), 65536) - prod
            near = Fraction(float(exact)) * 65536        # the subtraction's one rounding, then exact scaling
            assert got[j] == round(near), (j, dtype)


def test_out_of_range_steps_are_refused(net):
    w0 = stored(net)
    g = np.zeros(net.M)
    g[3] = 1.0
    assert not net.apply_gradient(g, 40000.0)          # one weight would pass -32768 pA
    assert not net.apply_gradient(np.full(net.M, np.nan), 1.0)
    assert np.array_equal(stored(net), w0)
    with pytest.raises(ValueError):
        net.apply_gradient(np.zeros(net.M + 1), 1.0)


def test_reset_restarts_the_trajectory_with_the_current_weights():
    """reset() returns to step 0 with the initial state: the run repeats bit
    for bit; after a weight change it equals a fresh network given the same
    weights by the same step."""
    w = tiny_adjoint_net()
    o = oracle.Oracle(w.to_dict())
    o.run(300)
    r0, y0 = o.raster(), o.state()
    o.reset()
    assert o.step == 0 and len(o.raster()[0]) == 0
    o.run(300)
    assert np.array_equal(o.raster()[1], r0[1]) and np.array_equal(o.state()[0], y0[0])
    g = np.full(o.M, 2.0)
    assert o.apply_gradient(g, 1.0)
    o.reset()
    o.run(300)
    f = oracle.Oracle(w.to_dict())
    assert f.apply_gradient(g, 1.0)
    f.run(300)
    assert np.array_equal(o.raster()[0], f.raster()[0]) and np.array_equal(o.raster()[1], f.raster()[1])
    assert np.array_equal(o.state()[0].view(np.uint64), f.state()[0].view(np.uint64))


def test_small_steps_against_the_gradient_lower_the_loss():
    """A small step against the adjoint gradient is a descent step: on a
    tiny network three such steps (window restarted from the initial state)
    lower the loss each time (a step along +g raises it: checked below)."""
    w = tiny_adjoint_net()
    o = oracle.Oracle(w.to_dict())
    losses = []
    eta = None
    for it in range(3):
        if it:
            o.reset()
        loss, g = o.adjoint(400, Y_STAR)
        losses.append(loss)
        if eta is None:
            eta = 1e-3 * loss / float(np.dot(g, g))
        assert o.apply_gradient(g, eta)
    assert losses[0] > losses[1] > losses[2], losses
    up = oracle.Oracle(w.to_dict())
    l0, g = up.adjoint(400, Y_STAR)
    assert up.apply_gradient(g, -eta)
    up.reset()
    assert up.adjoint(400, Y_STAR)[0] > l0
