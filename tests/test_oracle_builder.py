"""Pins of the oracle's network construction: exact structure, connection-rule
statistics, delay and weight laws, and byte equality with a brute-force
builder on tiny networks."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from naive_sim import Naive
from paper_2111_04398_amd import workloads


def tiny_fixed(seed=3):
    w = workloads.balanced(seed=seed)
    return w.replace(pop_size=[24, 8], conn=[[6.0, 2.0], [6.0, 2.0]], k_ext=[3000.0, 3000.0])


def tiny_bernoulli(seed=5):
    w = workloads.microcircuit(seed=seed)
    return w.replace(pop_size=[8, 3, 8, 3, 4, 2, 6, 2], conn=[[min(1.0, 2.5 * p) for p in r] for r in w.conn],
                     k_ext=[3000.0 + 100 * k for k in range(8)])


@pytest.fixture(scope="module")
def balanced_net():
    return oracle.Oracle(workloads.balanced().to_dict())


def test_fixed_indegree_exact_counts(balanced_net):
    """Every target has exactly 400 sources in [0, 4000) and 100 in [4000, 5000)."""
    rp, tg, w, d = balanced_net.synapses()
    N = balanced_net.N
    src = np.repeat(np.arange(N), np.diff(rp))
    exc = src < 4000
    assert np.array_equal(np.bincount(tg[exc], minlength=N), np.full(N, 400))
    assert np.array_equal(np.bincount(tg[~exc], minlength=N), np.full(N, 100))
    assert rp[-1] == 2_500_000


def test_fixed_indegree_outdegree_is_binomial(balanced_net):
    """With replacement, an E source's out-degree is Binomial(5000*400, 1/4000):
    mean 500, variance 499.875 (5 sigma on the sample moments); KS on the
    standardized degrees."""
    rp, *_ = balanced_net.synapses()
    deg = np.diff(rp)[:4000].astype(float)
    n, p = 5000 * 400, 1 / 4000
    mu, var = n * p, n * p * (1 - p)
    assert abs(deg.mean() - mu) < 5 * math.sqrt(var / 4000)
    assert abs(deg.var() - var) < 5 * var * math.sqrt(2 / 4000)
    degi = np.diff(rp)[4000:].astype(float)
    n, p = 5000 * 100, 1 / 1000
    assert abs(degi.mean() - n * p) < 5 * math.sqrt(n * p * (1 - p) / 1000)


def test_canonical_row_order(balanced_net):
    """Rows by source; within a row ascending target (multapses adjacent)."""
    rp, tg, *_ = balanced_net.synapses()
    for i in range(0, 5000, 97):
        row = tg[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) >= 0)


def _delay_pmf(mu_steps):
    """P(d = k) for d = clip(rint(N(mu, (mu/2)^2)), 1, 100) in steps."""
    sd = 0.5 * mu_steps
    ks = np.arange(1, 101)
    cdf = stats.norm.cdf
    p = cdf((ks + 0.5 - mu_steps) / sd) - cdf((ks - 0.5 - mu_steps) / sd)
    p[0] = cdf((1.5 - mu_steps) / sd)
    p[-1] = 1 - cdf((99.5 - mu_steps) / sd)
    return p


def test_delay_histogram_matches_discretised_normal(balanced_net):
    """Delays (steps) of E sources ~ rint(N(15, 7.5^2)) clipped to [1, 100], of
    I sources ~ rint(N(7.5, 3.75^2)) clipped; chi-square per class; every delay
    in [1, 100]."""
    rp, tg, w, d = balanced_net.synapses()
    src = np.repeat(np.arange(5000), np.diff(rp))
    assert d.min() >= 1 and d.max() <= 100
    for mask, mu in ((src < 4000, 15.0), (src >= 4000, 7.5)):
        obs = np.bincount(d[mask], minlength=101)[1:101].astype(float)
        exp = _delay_pmf(mu) * mask.sum()
        keep = exp > 20
        o = np.append(obs[keep], obs[~keep].sum())
        e = np.append(exp[keep], exp[~keep].sum())
        assert stats.chisquare(o, e * o.sum() / e.sum()).pvalue > 1e-4
    # P(d = 1) for E: Phi((1.5 - 15)/7.5) = 0.0359
    pe1 = (d[src < 4000] == 1).mean()
    assert abs(pe1 - 0.03593) < 5 * math.sqrt(0.0359 / (src < 4000).sum())


def test_weight_law(balanced_net):
    """w_q 2^-16 ~ N(87.8, 8.78^2) for E and N(-351.2, 35.12^2) for I sources,
    moments within 5 sigma, KS against the normal (quantisation 1.5e-5 pA is
    far below resolution)."""
    rp, tg, w, d = balanced_net.synapses()
    src = np.repeat(np.arange(5000), np.diff(rp))
    for mask, mu in ((src < 4000, 87.8), (src >= 4000, -351.2)):
        x = w[mask] * 2.0**-16
        n, sd = x.size, 0.1 * abs(mu)
        assert abs(x.mean() - mu) < 5 * sd / math.sqrt(n)
        assert abs(x.std() - sd) < 5 * sd / math.sqrt(2 * n)
        assert stats.kstest((x[:200000] - mu) / sd, "norm").pvalue > 1e-3


def test_weight_quantisation_of_one_synapse():
    """One synapse by hand: z from the oracle's Box-Muller of the W block,
    w = mu + 0.1|mu| z, w_q = rint(w 2^16) -- recomputed here in Python."""
    o = oracle.Oracle(workloads.balanced().to_dict(), synapses=False)
    for (a, b, post, pre) in ((17, 3, 0, 0), (4999, 499, 1, 1), (0, 0, 1, 0)):
        words = oracle.philox([a, b, 0, 4], [1, 0])
        z = oracle.box_muller(words)
        mu = 87.8 if pre == 0 else -351.2
        wq_expect = int(np.rint((mu + 0.1 * abs(mu) * z) * 65536.0))
        wq, d = o.weight_delay(a, b, post, pre)
        assert wq == wq_expect
        zd = oracle.box_muller(oracle.philox([a, b, 0, 5], [1, 0]))
        md = 1.5 if pre == 0 else 0.75
        assert d == min(max(int(np.rint((md + 0.5 * md * zd) / 0.1)), 1), 100)


@pytest.mark.parametrize("mk", [tiny_fixed, tiny_bernoulli])
def test_builder_equals_brute_force(mk):
    """Byte equality of the CSR store with the brute-force builder (numpy's
    Philox, pair/slot enumeration, Python floats)."""
    w = mk().to_dict()
    o = oracle.Oracle(w)
    nv = Naive(w)
    for a, b in zip(o.synapses(), nv.csr()):
        assert np.array_equal(a, b)


def test_bernoulli_counts_match_probabilities():
    """Pairwise Bernoulli at scale 0.1 of the microcircuit: per (post, pre)
    block the synapse count is Binomial(N_a N_b, floor(p 2^32)/2^32): z <= 5."""
    w = workloads.microcircuit(scale=0.1)
    o = oracle.Oracle(w.to_dict())
    rp, tg, *_ = o.synapses()
    off = o.pop_offsets()
    pop = np.searchsorted(off, np.arange(o.N), side="right") - 1
    src = np.repeat(np.arange(o.N), np.diff(rp))
    counts = np.zeros((8, 8))
    np.add.at(counts, (pop[tg], pop[src]), 1)
    sizes = np.diff(off)
    for a in range(8):
        for b in range(8):
            p = math.floor(w.conn[a][b] * 2**32) / 2**32
            n = sizes[a] * sizes[b]
            if p == 0:
                assert counts[a, b] == 0
                continue
            z = (counts[a, b] - n * p) / math.sqrt(n * p * (1 - p))
            assert abs(z) < 5, (a, b, z)
    # the per-row generator reproduces rows of the store
    for i in (0, 1, 2067, 5000, o.N - 1):
        assert np.array_equal(o.bernoulli_row(i), tg[rp[i]:rp[i + 1]])


def test_scaled_population_sizes():
    """Scale 0.1 of the microcircuit rounds to 7,717 neurons."""
    o = oracle.Oracle(workloads.microcircuit(scale=0.1).to_dict(), synapses=False)
    assert o.N == 7717
    assert list(np.diff(o.pop_offsets())) == [2068, 583, 2192, 548, 485, 106, 1440, 295]
