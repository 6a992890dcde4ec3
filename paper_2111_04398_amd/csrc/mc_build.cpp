// mc_build.cpp -- host-side network construction of libmc (C++17/OpenMP).
//
// Instantiation is outside the timed region (Methods: measurements start
// after model instantiation), so it runs on the host CPU cores.  Everything
// here is a deterministic function of the configuration: connection, weight,
// delay and initial-state draws are Philox blocks addressed by what they are
// for, and the transcendental functions are the C library's.
//
// Compile without FP contraction: weights and delays are rounded to integers
// after a few floating-point operations whose order is fixed.
#include "mc_build.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "mc_common.h"

namespace mc {
namespace {

struct Params {
  const mc_config* c;
  int n;                                 // populations
};

inline double param(const double* m, int n, int post, int pre) { return m[post * n + pre]; }

// One standard normal from the block keyed by (a, b, 0, tag): Box-Muller,
// cosine branch, from the first two words.
inline double normal_draw(uint64_t a, uint64_t b, uint64_t tag, uint64_t seed) {
  const U64x4 v = philox4x64_10(a, b, 0, tag, seed, 0);
  const double r = std::sqrt(-2.0 * std::log(u01_open_closed(v.w0)));
  return r * std::cos(6.283185307179586 * u01_closed_open(v.w1));
}

// Weight (2^-16 pA, round to nearest even) and delay (steps, clipped) of the
// synapse keyed (a, b).  Returns false if the weight does not fit int32.
inline bool weight_and_delay(const Params& p, uint64_t seed, uint64_t a, uint64_t b, int post, int pre,
                             int32_t& wq, uint8_t& d) {
  const mc_config& c = *p.c;
  const double mu = param(c.w_mean_pA, p.n, post, pre);
  const double w = mu + (c.w_rel_sd * std::fabs(mu)) * normal_draw(a, b, kTagW, seed);
  const double ws = w * 65536.0;
  if (!(std::fabs(ws) <= 2147483647.0)) return false;
  const long long q = std::llrint(ws);
  if (q > 2147483647LL || q < -2147483647LL) return false;
  const double md = c.d_mean_ms[pre];
  const double dms = md + (c.d_rel_sd * md) * normal_draw(a, b, kTagD, seed);
  long long s = std::llrint(dms / c.h_ms);
  s = std::min<long long>(std::max<long long>(s, c.d_min_steps), c.d_max_steps);
  wq = (int32_t)q;
  d = (uint8_t)s;
  return true;
}

struct Instance {
  int64_t N = 0;
  std::vector<int64_t> off;    // local population offsets [n+1]
  std::vector<uint8_t> pop;    // local
  uint64_t seed = 0;
};

// Pairwise Bernoulli rule: pass 1 counts each source row, pass 2 fills it.
// Both passes test the pair (i, j) against floor(p * 2^32) with the upper 32
// bits of word j&3 of the block keyed (i, j>>2, 0, CONN); the second pass
// recomputes the blocks instead of storing 6e9 outcomes.
bool build_bernoulli(const Params& p, const Instance& in, int64_t goff, HostNet& net, int64_t row0, int64_t m0,
                     std::vector<int64_t>& counts, bool fill, std::string& err) {
  const mc_config& c = *p.c;
  const int n = p.n;
  std::vector<uint64_t> thr((size_t)n * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const double pr = param(c.conn, n, a, b);
      thr[a * n + b] = (uint64_t)std::floor(pr * 4294967296.0);
    }
  const int64_t N = in.N;
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 32)
  for (int64_t i = 0; i < N; ++i) {
    const int b = in.pop[i];
    int64_t cnt = 0;
    int64_t pos = fill ? net.row_ptr[row0 + i] : 0;
    int64_t j = 0;
    for (int a = 0; a < n; ++a) {
      const uint64_t T = thr[a * n + b];
      const int64_t jend = in.off[a + 1];
      if (T == 0) { j = jend; continue; }
      for (; j < jend; ++j) {
        // one Philox block per aligned quad of targets
        const U64x4 v = philox4x64_10((uint64_t)i, (uint64_t)(j >> 2), 0, kTagConn, in.seed, 0);
        const uint64_t u = hi32(pick(v, (unsigned)(j & 3)));
        if (u < T) {
          if (fill) {
            net.tgt[pos] = (int32_t)(goff + j);
            if (!weight_and_delay(p, in.seed, (uint64_t)i, (uint64_t)j, a, b, net.wq[pos], net.dly[pos])) ok = false;
            ++pos;
          }
          ++cnt;
        }
      }
    }
    if (!fill) counts[i] = cnt;
  }
  (void)m0;
  if (!ok) err = "a quantised weight does not fit in int32";
  return ok;
}

}  // namespace

static int fail(std::string& err, int code, const char* msg) { err = msg; return code; }

// Connections of one Bernoulli instance from a connection builder, then the
// weight and delay of every synapse on the host (the draws keyed (i, j) that
// the host's own pass 2 makes).
static int build_bernoulli_with(const Params& p, const Instance& in, int64_t goff, HostNet& net, ConnBuilder& conn,
                         const std::vector<uint64_t>& thr, std::vector<int64_t>& counts, bool fill, std::string& err) {
  BernoulliPlan plan;
  plan.N = in.N;
  plan.n_pops = p.n;
  plan.off = in.off.data();
  plan.pop = in.pop.data();
  plan.thr = thr.data();
  plan.seed = in.seed;
  plan.goff = goff;
  if (!fill) return conn.count(plan, counts.data(), err);
  const int64_t base = net.row_ptr[goff];
  std::vector<int64_t> rp((size_t)in.N + 1);
  for (int64_t i = 0; i <= in.N; ++i) rp[i] = net.row_ptr[goff + i] - base;
  int rc = conn.fill(plan, rp.data(), net.tgt.data() + base, err);
  if (rc != MC_OK) return rc;
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 32) reduction(&& : ok)
  for (int64_t i = 0; i < in.N; ++i)
    for (int64_t e = base + rp[i]; e < base + rp[i + 1]; ++e) {
      const int64_t j = net.tgt[e] - goff;
      if (!weight_and_delay(p, in.seed, (uint64_t)i, (uint64_t)j, in.pop[j], in.pop[i], net.wq[e], net.dly[e])) ok = false;
    }
  if (!ok) { err = "a quantised weight does not fit in int32"; return MC_ERR_RANGE; }
  return MC_OK;
}

static std::vector<uint64_t> bernoulli_thresholds(const mc_config& c, int n) {
  std::vector<uint64_t> thr((size_t)n * n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) thr[a * n + b] = (uint64_t)std::floor(param(c.conn, n, a, b) * 4294967296.0);
  return thr;
}

int build_host(const mc_config& c, HostNet& net, std::string& err, ConnBuilder* conn) {
  if (c.struct_size != sizeof(mc_config)) return fail(err, MC_ERR_INVALID_ARG, "mc_config.struct_size mismatch");
  const int n = c.n_pops;
  if (n < 1 || n > kMaxPops) return fail(err, MC_ERR_INVALID_ARG, "n_pops must be in [1, 16]");
  if (!c.pop_size || !c.conn || !c.w_mean_pA || !c.d_mean_ms || !c.k_ext)
    return fail(err, MC_ERR_INVALID_ARG, "NULL population array");
  if (c.n_instances < 1 || !c.inst_seed) return fail(err, MC_ERR_INVALID_ARG, "n_instances >= 1 and inst_seed required");
  if (c.rule != MC_RULE_FIXED_INDEGREE && c.rule != MC_RULE_BERNOULLI) return fail(err, MC_ERR_INVALID_ARG, "unknown rule");
  if (!(c.h_ms > 0) || !(c.tau_m_ms > 0) || !(c.tau_syn_ms > 0) || !(c.c_m_pF > 0))
    return fail(err, MC_ERR_INVALID_ARG, "h, tau_m, tau_syn and C_m must be positive");
  if (c.tau_m_ms == c.tau_syn_ms) return fail(err, MC_ERR_INVALID_ARG, "tau_m == tau_syn (singular propagator) unsupported");
  if (c.d_min_steps < 1 || c.d_max_steps < c.d_min_steps || c.d_max_steps > 100)
    return fail(err, MC_ERR_RANGE, "delays must satisfy 1 <= d_min <= d_max <= 100 steps");
  if (!(c.t_ref_ms >= 0)) return fail(err, MC_ERR_INVALID_ARG, "t_ref must be >= 0");
  if (!(c.nu_ext_hz >= 0) || !(c.w_rel_sd >= 0) || !(c.d_rel_sd >= 0)) return fail(err, MC_ERR_INVALID_ARG, "negative rate or spread");
  if (!(c.v0_hi_mV >= c.v0_lo_mV)) return fail(err, MC_ERR_INVALID_ARG, "v0_hi < v0_lo");
  for (int a = 0; a < n; ++a) {
    if (c.pop_size[a] < 1) return fail(err, MC_ERR_INVALID_ARG, "population sizes must be >= 1");
    if (!(c.k_ext[a] >= 0)) return fail(err, MC_ERR_INVALID_ARG, "k_ext must be >= 0");
    if (!(c.d_mean_ms[a] >= 0)) return fail(err, MC_ERR_INVALID_ARG, "d_mean must be >= 0");
    for (int b = 0; b < n; ++b) {
      const double v = c.conn[a * n + b];
      if (c.rule == MC_RULE_BERNOULLI && !(v >= 0.0 && v <= 1.0)) return fail(err, MC_ERR_INVALID_ARG, "probability outside [0, 1]");
      if (c.rule == MC_RULE_FIXED_INDEGREE && !(v >= 0.0 && v <= 1e6)) return fail(err, MC_ERR_INVALID_ARG, "in-degree outside [0, 1e6]");
    }
  }
  const long long ref = std::llrint(c.t_ref_ms / c.h_ms);
  if (ref > 255) return fail(err, MC_ERR_RANGE, "t_ref / h above 255 steps");

  Params p{&c, n};
  net.n_pops = n;
  net.n_inst = c.n_instances;
  // instance sizes
  std::vector<Instance> inst((size_t)c.n_instances);
  net.inst_off.assign((size_t)c.n_instances + 1, 0);
  net.pop_off.assign((size_t)c.n_instances * (n + 1), 0);
  net.inst_seed.resize(c.n_instances);
  net.inst_scale.resize(c.n_instances);
  for (int b = 0; b < c.n_instances; ++b) {
    Instance& in = inst[b];
    const double s = c.inst_scale ? c.inst_scale[b] : 1.0;
    if (!(s > 0)) return fail(err, MC_ERR_INVALID_ARG, "instance scale must be positive");
    in.seed = c.inst_seed[b];
    in.off.assign(n + 1, 0);
    for (int a = 0; a < n; ++a) {
      long long sz = std::llrint(s * (double)c.pop_size[a]);
      if (sz < 1) sz = 1;
      in.off[a + 1] = in.off[a] + sz;
    }
    in.N = in.off[n];
    in.pop.resize((size_t)in.N);
    for (int a = 0; a < n; ++a) std::fill(in.pop.begin() + in.off[a], in.pop.begin() + in.off[a + 1], (uint8_t)a);
    net.inst_off[b + 1] = net.inst_off[b] + in.N;
    for (int a = 0; a <= n; ++a) net.pop_off[(size_t)b * (n + 1) + a] = net.inst_off[b] + in.off[a];
    net.inst_seed[b] = in.seed;
    net.inst_scale[b] = s;
  }
  net.N = net.inst_off[c.n_instances];
  if (net.N >= (int64_t)1 << 30) return fail(err, MC_ERR_RANGE, "more than 2^30 neurons");
  net.pop_of.resize((size_t)net.N);
  for (int b = 0; b < c.n_instances; ++b)
    std::memcpy(net.pop_of.data() + net.inst_off[b], inst[b].pop.data(), (size_t)inst[b].N);

  // propagators of the exact integration step (matrix exponential of the
  // linear subthreshold system over h)
  const double h = c.h_ms;
  net.P22 = std::exp(-h / c.tau_m_ms);
  net.P11 = std::exp(-h / c.tau_syn_ms);
  net.P21 = ((c.tau_syn_ms * c.tau_m_ms) / (c.c_m_pF * (c.tau_m_ms - c.tau_syn_ms))) * (net.P22 - net.P11);
  net.P20 = -(c.tau_m_ms / c.c_m_pF) * std::expm1(-h / c.tau_m_ms);
  net.i_e = c.i_e_pA;
  net.theta = c.v_th_mV - c.e_l_mV;
  net.y_reset = c.v_reset_mV - c.e_l_mV;
  net.e_l = c.e_l_mV;
  net.ref_steps = (int)ref;
  {
    const double jq = c.w_ext_pA * 65536.0;
    if (!(std::fabs(jq) <= 2147483647.0)) return fail(err, MC_ERR_RANGE, "w_ext does not fit the fixed-point format");
    net.jext_q = std::llrint(jq);
  }
  // Poisson inverse CDF per population: T[k] = min(floor(F(k) 2^32), 2^32),
  // T[63] = 2^32, F accumulated from p_k = p_{k-1} * lambda / k.
  net.table.assign((size_t)n * kTableLen, 0);
  for (int a = 0; a < n; ++a) {
    const double lam = ((c.nu_ext_hz * c.k_ext[a]) * h) * 1e-3;
    double pk = std::exp(-lam), F = pk;
    for (int k = 0; k < kTableLen; ++k) {
      if (k > 0) { pk = pk * lam / (double)k; F = F + pk; }
      const double t = std::floor(F * 4294967296.0);
      net.table[(size_t)a * kTableLen + k] = t >= 4294967296.0 ? 4294967296ULL : (uint64_t)t;
    }
    net.table[(size_t)a * kTableLen + kTableLen - 1] = 4294967296ULL;
  }
  // initial membrane potentials: uniform in [v0_lo, v0_hi)
  net.y0.resize((size_t)net.N);
  for (int b = 0; b < c.n_instances; ++b) {
    const Instance& in = inst[b];
    const int64_t g = net.inst_off[b];
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < (in.N + 3) / 4; ++q) {
      const U64x4 v = philox4x64_10((uint64_t)q, 0, 0, kTagV0, in.seed, 0);
      for (int k = 0; k < 4; ++k) {
        const int64_t i = 4 * q + k;
        if (i >= in.N) break;
        net.y0[g + i] = (c.v0_hi_mV - c.v0_lo_mV) * u01_closed_open(pick(v, k)) + (c.v0_lo_mV - c.e_l_mV);
      }
    }
  }

  // synapses, instance by instance (block-diagonal)
  net.row_ptr.assign((size_t)net.N + 1, 0);
  if (c.rule == MC_RULE_BERNOULLI) {
    std::vector<std::vector<int64_t>> counts((size_t)c.n_instances);
    const std::vector<uint64_t> thr = bernoulli_thresholds(c, n);
    for (int b = 0; b < c.n_instances; ++b) {
      counts[b].assign((size_t)inst[b].N, 0);
      if (conn) {
        const int rc = build_bernoulli_with(p, inst[b], net.inst_off[b], net, *conn, thr, counts[b], false, err);
        if (rc != MC_OK) return rc;
      } else {
        build_bernoulli(p, inst[b], net.inst_off[b], net, net.inst_off[b], 0, counts[b], false, err);
      }
      for (int64_t i = 0; i < inst[b].N; ++i)
        net.row_ptr[net.inst_off[b] + i + 1] = net.row_ptr[net.inst_off[b] + i] + counts[b][i];
      if (b + 1 < c.n_instances) net.row_ptr[net.inst_off[b + 1]] = net.row_ptr[net.inst_off[b] + inst[b].N];
    }
    net.M = net.row_ptr[net.N];
    try {
      net.tgt.resize((size_t)net.M); net.wq.resize((size_t)net.M); net.dly.resize((size_t)net.M);
    } catch (...) { return fail(err, MC_ERR_OOM, "host allocation of the synapse store failed"); }
    for (int b = 0; b < c.n_instances; ++b) {
      if (conn) {
        const int rc = build_bernoulli_with(p, inst[b], net.inst_off[b], net, *conn, thr, counts[b], true, err);
        if (rc != MC_OK) return rc;
      } else if (!build_bernoulli(p, inst[b], net.inst_off[b], net, net.inst_off[b], 0, counts[b], true, err)) {
        return MC_ERR_RANGE;
      }
    }
  } else {
    // Fixed in-degree: target j draws, for each presynaptic population in
    // order, conn[a][b] sources uniformly with replacement; draw m of target j
    // uses word m&3 of the block keyed (j, m>>2, 0, SRC).  The store is the
    // stable counting sort of the (j, m) list by source.
    for (int b = 0; b < c.n_instances; ++b) {
      const Instance& in = inst[b];
      const int64_t g = net.inst_off[b];
      std::vector<int64_t> K((size_t)n * n);
      std::vector<int64_t> kin(n, 0);   // in-degree of a target in population a
      for (int a = 0; a < n; ++a)
        for (int bb = 0; bb < n; ++bb) { K[a * n + bb] = std::llrint(c.conn[a * n + bb]); kin[a] += K[a * n + bb]; }
      std::vector<int64_t> first((size_t)in.N + 1, 0);   // offset of target j's draws
      for (int64_t j = 0; j < in.N; ++j) first[j + 1] = first[j] + kin[in.pop[j]];
      const int64_t Mb = first[in.N];
      std::vector<int32_t> src((size_t)Mb);
      if (conn) {
        FixedPlan plan;
        plan.N = in.N;
        plan.n_pops = n;
        plan.off = in.off.data();
        plan.pop = in.pop.data();
        plan.K = K.data();
        plan.first = first.data();
        plan.seed = in.seed;
        const int rc = conn->sources(plan, src.data(), err);
        if (rc != MC_OK) return rc;
      } else {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t j = 0; j < in.N; ++j) {
          const int a = in.pop[j];
          int64_t m = 0;
          for (int bb = 0; bb < n; ++bb) {
            const uint64_t Nb = (uint64_t)(in.off[bb + 1] - in.off[bb]);
            for (int64_t q = 0; q < K[a * n + bb]; ++q, ++m) {
              const U64x4 v = philox4x64_10((uint64_t)j, (uint64_t)(m >> 2), 0, kTagSrc, in.seed, 0);
              const uint64_t u = hi32(pick(v, (unsigned)(m & 3)));
              src[first[j] + m] = (int32_t)(in.off[bb] + (int64_t)((u * Nb) >> 32));
            }
          }
        }
      }
      std::vector<int64_t> cnt((size_t)in.N + 1, 0);
      for (int64_t e = 0; e < Mb; ++e) cnt[src[e] + 1]++;
      for (int64_t i = 0; i < in.N; ++i) cnt[i + 1] += cnt[i];
      const int64_t base = net.row_ptr[g];
      for (int64_t i = 0; i < in.N; ++i) net.row_ptr[g + i + 1] = base + cnt[i + 1];
      net.M = base + Mb;
      try {
        net.tgt.resize((size_t)net.M); net.wq.resize((size_t)net.M); net.dly.resize((size_t)net.M);
      } catch (...) { return fail(err, MC_ERR_OOM, "host allocation of the synapse store failed"); }
      std::vector<int64_t> slot_of((size_t)Mb);    // draw index m of each stored synapse
      std::vector<int64_t> fillpos(cnt.begin(), cnt.end() - 1);
      for (int64_t j = 0; j < in.N; ++j)
        for (int64_t m = 0; m < first[j + 1] - first[j]; ++m) {
          const int64_t pos = fillpos[src[first[j] + m]]++;
          net.tgt[base + pos] = (int32_t)(g + j);
          slot_of[pos] = m;
        }
      bool ok = true;
#pragma omp parallel for schedule(dynamic, 64) reduction(&& : ok)
      for (int64_t i = 0; i < in.N; ++i) {
        for (int64_t e = cnt[i]; e < cnt[i + 1]; ++e) {
          const int64_t j = net.tgt[base + e] - g;
          if (!weight_and_delay(p, in.seed, (uint64_t)j, (uint64_t)slot_of[e], in.pop[j], in.pop[i],
                                net.wq[base + e], net.dly[base + e])) ok = false;
        }
      }
      if (!ok) return fail(err, MC_ERR_RANGE, "a quantised weight does not fit in int32");
    }
  }
  int64_t mx = 0;
  for (int64_t i = 0; i < net.N; ++i) mx = std::max(mx, net.row_ptr[i + 1] - net.row_ptr[i]);
  if (mx > (int64_t)1 << 30) return fail(err, MC_ERR_RANGE, "row longer than 2^30 synapses");
  net.max_row = (int)mx;
  int dm = 0;
#pragma omp parallel for reduction(max : dm)
  for (int64_t e = 0; e < net.M; ++e) dm = std::max(dm, (int)net.dly[e]);
  net.max_delay = dm;
  return MC_OK;
}

}  // namespace mc
