"""Pins of the oracle's propagators and Poisson drive tables against
high-precision closed forms and the Poisson law."""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2111_04398_amd import workloads

mpmath.mp.dps = 40


def ulp_err(x: float, exact) -> float:
    return float(abs(mpmath.mpf(x) - exact) / mpmath.mpf(math.ulp(x)))


def test_propagators_match_40_digit_closed_form():
    """Exact integration of dy/dt = -y/tau_m + I/C, dI/dt = -I/tau_s over h:
    P22 = e^{-h/tau_m}, P11 = e^{-h/tau_s},
    P21 = tau_s tau_m / (C (tau_m - tau_s)) (P22 - P11), P20 = tau_m/C (1 - P22);
    values from mpmath at 40 digits.  P11, P22: one correctly rounded libm
    call each (<= 1 ulp).  P21: the difference P22 - P11 is exact (Sterbenz)
    but carries both inputs' half-ulp errors (1.1e-16 absolute on 0.171), so
    with the prefactor's rounding the bound is about 5 ulp of P21.  P20: expm1
    plus one product, <= 2 ulp."""
    o = oracle.Oracle(workloads.balanced().to_dict(), synapses=False)
    P11, P21, P22, P20 = o.propagators()
    h, tm, ts, C = (mpmath.mpf(v) for v in ("0.1", "10", "0.5", "250"))
    e22, e11 = mpmath.exp(-h / tm), mpmath.exp(-h / ts)
    assert ulp_err(P22, e22) <= 1.0
    assert ulp_err(P11, e11) <= 1.0
    assert ulp_err(P21, ts * tm / (C * (tm - ts)) * (e22 - e11)) <= 5.0
    assert ulp_err(P20, tm / C * (1 - e22)) <= 2.0
    # printed digits, as a second, literal pin
    assert P22 == pytest.approx(0.990049833749168053574, rel=2e-16)
    assert P11 == pytest.approx(0.818730753077981858670, rel=2e-16)
    assert P21 == pytest.approx(3.60671748781444621e-4, rel=5e-16)
    assert P20 == pytest.approx(3.98006650033277857e-4, rel=5e-16)


@pytest.mark.parametrize("lam_kext", [1000.0, 1500.0, 2100.0, 2900.0, 0.0])
def test_poisson_table_is_inverse_cdf(lam_kext):
    """Table entry k = min(floor(F(k) 2^32), 2^32), last entry 2^32: it is
    non-decreasing and (T_k - T_{k-1}) / 2^32 equals the Poisson pmf of
    lambda = nu K h within 2^-32 + 1e-15 (pmf from mpmath)."""
    w = workloads.balanced().replace(k_ext=[lam_kext, lam_kext])
    o = oracle.Oracle(w.to_dict(), synapses=False)
    T = o.tables()[0].astype(object)
    lam = mpmath.mpf(8) * mpmath.mpf(lam_kext) * mpmath.mpf("0.1") * mpmath.mpf("1e-3")
    assert all(T[k] <= T[k + 1] for k in range(63))
    assert T[63] == 2**32
    prev = 0
    for k in range(40):
        pk = mpmath.exp(-lam) * lam**k / mpmath.factorial(k)
        got = mpmath.mpf(int(T[k]) - prev) / 2**32
        assert abs(got - pk) <= mpmath.mpf(2) ** -32 + mpmath.mpf("1e-15"), k
        prev = int(T[k])


def test_poisson_draws_have_poisson_moments():
    """Counts drawn by the oracle over 4e5 (neuron, step) pairs: mean and
    variance equal lambda = 0.8 within 5 sigma; chi-square against the pmf."""
    w = workloads.balanced().replace(pop_size=[400, 100])
    o = oracle.Oracle(w.to_dict(), synapses=False)
    ks = np.array([o.poisson_count(s, i) for s in range(800) for i in range(500)])
    lam, n = 0.8, ks.size
    assert abs(ks.mean() - lam) < 5 * math.sqrt(lam / n)
    assert abs(ks.var() - lam) < 5 * math.sqrt((lam + 2 * lam * lam) / n)
    obs = np.bincount(ks, minlength=8)[:6]
    exp = stats.poisson.pmf(np.arange(6), lam) * n
    obs = np.append(obs, n - obs.sum())
    exp = np.append(exp, n - exp.sum())
    assert stats.chisquare(obs, exp).pvalue > 1e-3


def test_external_weight_quantisation():
    """J = 87.8 pA in units of 2^-16 pA, rounded to nearest: 5,754,061."""
    o = oracle.Oracle(workloads.balanced().to_dict(), synapses=False)
    assert o.jext_q() == 5754061


def _golden_parameters():
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_parameters.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            name, value = line.split()[:2]
            out[name] = float(value)
    return out


def test_paper_parameters_golden():
    """The microcircuit workload and the oracle's propagators use what the
    paper prints (tests/golden/paper_parameters.txt): h, the smallest delay,
    tau_syn, tau_m, 10 s after a 0.1 s presimulation, about 8e4 neurons in
    8 populations and about 3e8 synapses (expected count of the pairwise
    rule, within 5 %)."""
    g = _golden_parameters()
    w = workloads.microcircuit()
    assert w.h == g["h"] and w.tau_syn == g["tau_syn"] and w.tau_m == g["tau_m"]
    assert w.d_min_steps * w.h == pytest.approx(g["d_min"])
    assert w.sim_steps * w.h * 1e-3 == pytest.approx(g["t_model"])
    assert w.presim_steps * w.h * 1e-3 == pytest.approx(g["t_presim"])
    assert w.n_pops == g["populations"]
    N = np.asarray(w.pop_size, float)
    assert abs(N.sum() / g["neurons"] - 1) < 0.05
    p = np.floor(np.asarray(w.conn, float) * 2.0**32) / 2.0**32      # [post][pre]
    expected_m = float((p * N[:, None] * N[None, :]).sum())
    assert abs(expected_m / g["synapses"] - 1) < 0.05
    o = oracle.Oracle(w.to_dict(), synapses=False)
    P11, _, P22, _ = o.propagators()
    assert P22 == math.exp(-g["h"] / g["tau_m"]) and P11 == math.exp(-g["h"] / g["tau_syn"])
