"""Pins of the oracle's random-number layer against numpy and the normal law."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from naive_sim import philox_np
from paper_2111_04398_amd import workloads


def test_philox_matches_numpy_random_counters():
    """Philox4x64-10 (Salmon et al. 2011) against numpy's independent
    implementation on random counters/keys, including counters whose low word
    is zero (the numpy pre-increment then borrows across words)."""
    rng = np.random.default_rng(7)
    n = 2000
    ctr = rng.integers(0, 2**63, size=(n, 4), dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=(n, 4), dtype=np.uint64)
    ctr[:50, 0] = 0
    ctr[50:60, :3] = 0
    key = rng.integers(0, 2**63, size=(n, 2), dtype=np.uint64) * np.uint64(2)
    got = oracle.philox_many(ctr, key)
    for k in range(n):
        c = [int(v) for v in ctr[k]]
        ref = philox_np(c[0], c[1], c[2], c[3], int(key[k, 0]), int(key[k, 1]))
        assert [int(v) for v in got[k]] == ref, k


def test_philox_bulk_against_numpy_stream():
    """A numpy Philox stream of 10^6 words (consecutive counters) equals the
    oracle's blocks at counters 1, 2, ..."""
    key = np.array([0x1234567890ABCDEF, 42], np.uint64)
    bg = np.random.Philox(counter=np.zeros(4, np.uint64), key=key)
    stream = bg.random_raw(4 * 250000).reshape(-1, 4)
    ctr = np.zeros((250000, 4), np.uint64)
    ctr[:, 0] = np.arange(1, 250001, dtype=np.uint64)
    got = oracle.philox_many(ctr, np.tile(key, (250000, 1)))
    assert np.array_equal(got, stream)


def test_box_muller_is_standard_normal():
    """z from the cosine branch of Box-Muller: KS test against N(0, 1) and
    moments within 5 sigma over 2e5 draws."""
    n = 200000
    ctr = np.zeros((n, 4), np.uint64)
    ctr[:, 0] = np.arange(n, dtype=np.uint64)
    ctr[:, 3] = 4
    words = oracle.philox_many(ctr, np.tile(np.array([3, 0], np.uint64), (n, 1)))
    z = np.array([oracle.box_muller(words[k]) for k in range(n)])
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_box_muller_formula_on_known_words():
    """The transform on hand-picked words: u1 = ((w0>>11)+1) 2^-53 in (0, 1],
    u2 = (w1>>11) 2^-53 in [0, 1)."""
    top = (1 << 64) - 1
    # u1 = 1 -> radius 0
    assert oracle.box_muller(np.array([top, 5, 0, 0], np.uint64)) == 0.0
    # u1 = 2^-53 (smallest), u2 = 0 -> sqrt(-2 ln 2^-53)
    z = oracle.box_muller(np.array([0, 0, 0, 0], np.uint64))
    assert z == pytest.approx(math.sqrt(2 * 53 * math.log(2)), rel=1e-15)
    # u2 = 1/2 -> cos(pi) = -1
    z = oracle.box_muller(np.array([(1 << 63) - 1, 1 << 63, 0, 0], np.uint64))
    assert z == pytest.approx(-math.sqrt(-2 * math.log(0.5)), rel=1e-15)


def test_instance_scales_match_input_generator():
    """The batched instance scales drawn by the oracle equal the ones the
    workload generator draws with numpy's Philox, and lie in [0.05, 0.25)."""
    s_np = workloads.batch_scales(64)
    s_or = [oracle.instance_scale(b) for b in range(64)]
    assert s_np == s_or
    assert min(s_np) >= 0.05 and max(s_np) < 0.25
