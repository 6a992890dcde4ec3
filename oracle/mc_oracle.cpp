// mc_oracle.cpp -- plain CPU oracle for the microcircuit simulation cycle.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no source, header, table or helper with the HIP
// path: it has its own Philox, its own network builder, its own propagators
// and its own simulation loop, written for obviousness, not speed.
//
// What it computes (Kurth et al., "Sub-realtime simulation of a neuronal
// network of natural density"):
//   * the simulation cycle of the Methods section / Fig. 1b caption: "update"
//     integrates every neuron's state by one step of h = 0.1 ms, "deliver"
//     distributes each spike through the explicitly stored synapses of its
//     source into delay-indexed input buffers (Supplementary Fig. 1 caption:
//     h = 0.1 ms, smallest delay 0.1 ms, tau_syn = 0.5 ms, tau_m = 10 ms);
//   * the neuron is the leaky integrate-and-fire neuron with exponentially
//     decaying synaptic current, advanced by exact integration of its linear
//     subthreshold dynamics (the closed-form propagator of a linear ODE over
//     one step), with threshold, reset and refractoriness;
//   * weights are stored explicitly per synapse (Discussion), here as signed
//     fixed-point integers in units of 2^-16 pA so that every input sum is an
//     exact integer sum, independent of summation order;
//   * external drive is a Poisson count per neuron and step drawn by inverting
//     the Poisson CDF with one 32-bit uniform from a counter-based generator;
//   * the reverse-time adjoint of a membrane-potential loss with the spike
//     pattern held fixed (Discussion: plasticity and learning are possible in
//     this explicit-synapse representation), and a quad-precision finite
//     difference of the same loss.
// The paper prints no equations beyond the realtime factor; every reading of
// it that this file fixes is listed in the design notes beside the package.
//
// Build: g++ -O2 -fopenmp -ffp-contract=off -fno-fast-math -fPIC -shared
// (floating point: IEEE double, no contraction, libm for exp/expm1/log/cos/sqrt).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdio>
#include <vector>
#include <algorithm>
#include <numeric>
#include <chrono>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
// as 1, 2, 3", SC'11).  Ten rounds; each round multiplies counter words 0 and
// 2 by the published multipliers, and the key is bumped by the published Weyl
// increments between rounds.
// ---------------------------------------------------------------------------
const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL;
const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL;

struct Word4 { uint64_t v[4]; };

Word4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1) {
  uint64_t c[4] = {c0, c1, c2, c3};
  uint64_t k[2] = {k0, k1};
  for (int round = 0; round < 10; ++round) {
    if (round > 0) { k[0] += PHILOX_W0; k[1] += PHILOX_W1; }
    unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c[0];
    unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c[2];
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c[1] ^ k[0];
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c[3] ^ k[1];
    uint64_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  Word4 w; for (int i = 0; i < 4; ++i) w.v[i] = c[i];
  return w;
}

// Stream tags (last counter word): which random quantity a draw belongs to.
enum { TAG_V0 = 1, TAG_CONN = 2, TAG_SRC = 3, TAG_W = 4, TAG_D = 5, TAG_DRIVE = 6, TAG_SCALE = 7 };

inline uint32_t upper32(uint64_t w) { return (uint32_t)(w >> 32); }
inline double unit53(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }            // [0, 1)
inline double unit53_open0(uint64_t w) { return (double)((w >> 11) + 1) * 0x1p-53; } // (0, 1]

// Standard normal by the Box-Muller transform (cosine branch only), from the
// two first words of one Philox block.
double box_muller(const Word4& w) {
  double u1 = unit53_open0(w.v[0]);
  double u2 = unit53(w.v[1]);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

}  // namespace

// ---------------------------------------------------------------------------
// Configuration (the oracle's own; nothing is shared with the library header)
// ---------------------------------------------------------------------------
extern "C" {

#define ORC_MAXPOP 16

typedef struct orc_cfg {
  int32_t n_pops;
  int32_t pop_size[ORC_MAXPOP];     // before scaling
  int32_t pop_is_exc[ORC_MAXPOP];
  int32_t rule;                     // 0: fixed in-degree, 1: pairwise Bernoulli
  double conn[ORC_MAXPOP * ORC_MAXPOP];    // [post*n_pops+pre]: in-degree or probability
  double w_mean[ORC_MAXPOP * ORC_MAXPOP];  // [post*n_pops+pre], pA, signed
  double w_rel_sd;
  double d_mean[ORC_MAXPOP];        // per presynaptic population, ms
  double d_rel_sd;
  int32_t d_min_steps, d_max_steps;
  double k_ext[ORC_MAXPOP];         // external in-degree per population
  double nu_ext;                    // Hz
  double w_ext;                     // pA
  double tau_m, c_m, e_l, v_reset, v_th, t_ref, tau_syn, i_e, h;
  double v0_lo, v0_hi;
  uint64_t seed;
  double scale;                     // population sizes become max(1, rint(scale*size))
} orc_cfg;

}  // extern "C"

namespace {

struct Net {
  orc_cfg cfg;
  int n_pops = 0;
  std::vector<int64_t> pop_off;   // n_pops+1
  std::vector<int32_t> pop_of;    // N
  int64_t N = 0;
  // source-major synapse store, canonical order
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> tgt;
  std::vector<int32_t> wq;
  std::vector<uint8_t> dly;
  // propagators and drive
  double P11 = 0, P21 = 0, P22 = 0, P20 = 0;
  std::vector<uint64_t> table;    // [n_pops][64]
  int64_t jext_q = 0;
  int ref_steps = 0;
  double theta = 0, y_reset = 0;
  // state
  std::vector<double> y, I;
  std::vector<int32_t> r;
  int D = 0;                      // ring depth = d_max + 1
  std::vector<std::vector<int64_t>> ring;  // [D][N]
  int64_t step = 0;
  std::vector<int32_t> raster_step, raster_id;
  std::vector<int64_t> spikes_per_pop;
  int64_t events = 0;
  int err = 0;
};

int64_t scaled_size(double scale, int32_t n) {
  long long v = std::llrint(scale * (double)n);
  return v < 1 ? 1 : v;
}

// Exact integration of the subthreshold dynamics over one step h:
//   dy/dt = -y/tau_m + I/C_m,  dI/dt = -I/tau_syn  (y = V - E_L)
// gives y' = P22*y + P21*I + P20*I_e and I' = P11*I, with the propagators
// below (matrix exponential of the linear system).
void make_propagators(Net& n) {
  const orc_cfg& c = n.cfg;
  n.P22 = std::exp(-c.h / c.tau_m);
  n.P11 = std::exp(-c.h / c.tau_syn);
  n.P21 = ((c.tau_syn * c.tau_m) / (c.c_m * (c.tau_m - c.tau_syn))) * (n.P22 - n.P11);
  n.P20 = -(c.tau_m / c.c_m) * std::expm1(-c.h / c.tau_m);
}

// Inverse-CDF table of the Poisson count per step with mean
// lambda = nu * K_ext * h: entry k is floor(F(k) * 2^32), capped at 2^32, and
// the last entry is forced to 2^32 so every 32-bit uniform maps to a count.
void make_table(Net& n) {
  const orc_cfg& c = n.cfg;
  n.table.assign((size_t)n.n_pops * 64, 0);
  for (int p = 0; p < n.n_pops; ++p) {
    double lambda = ((c.nu_ext * c.k_ext[p]) * c.h) * 1e-3;
    double pk = std::exp(-lambda);
    double F = pk;
    for (int k = 0; k < 64; ++k) {
      if (k > 0) { pk = pk * lambda / (double)k; F = F + pk; }
      double scaled = std::floor(F * 4294967296.0);
      uint64_t T = scaled >= 4294967296.0 ? 4294967296ULL : (uint64_t)scaled;
      n.table[(size_t)p * 64 + k] = T;
    }
    n.table[(size_t)p * 64 + 63] = 4294967296ULL;
  }
}

// Weight and delay of one synapse, from the normal draws keyed by (a, b).
bool draw_weight_delay(const Net& n, uint64_t a, uint64_t b, int post, int pre,
                       int32_t* wq_out, uint8_t* d_out) {
  const orc_cfg& c = n.cfg;
  uint64_t seed = c.seed;
  double mu = c.w_mean[post * n.n_pops + pre];
  double zw = box_muller(philox(a, b, 0, TAG_W, seed, 0));
  double w = mu + (c.w_rel_sd * std::fabs(mu)) * zw;
  double wscaled = w * 65536.0;
  if (!(std::fabs(wscaled) <= 2147483647.0)) return false;
  long long q = std::llrint(wscaled);
  if (q > 2147483647LL || q < -2147483647LL) return false;
  double md = c.d_mean[pre];
  double zd = box_muller(philox(a, b, 0, TAG_D, seed, 0));
  double dms = md + (c.d_rel_sd * md) * zd;
  long long d = std::llrint(dms / c.h);
  if (d < c.d_min_steps) d = c.d_min_steps;
  if (d > c.d_max_steps) d = c.d_max_steps;
  *wq_out = (int32_t)q;
  *d_out = (uint8_t)d;
  return true;
}

struct Syn { int64_t src; int32_t tgt; int32_t slot; int32_t wq; uint8_t d; };

// Fixed in-degree: every target j draws, for each presynaptic population b in
// order, conn[a][b] sources uniformly from b with replacement (autapses and
// multapses allowed).  Slot m numbers the draws of target j.
bool build_fixed_indegree(Net& n) {
  const orc_cfg& c = n.cfg;
  std::vector<std::vector<Syn>> per_target((size_t)n.N);
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 64) reduction(&& : ok)
  for (int64_t j = 0; j < n.N; ++j) {
    int a = n.pop_of[j];
    int64_t m = 0;
    for (int b = 0; b < n.n_pops; ++b) {
      long long K = std::llrint(c.conn[a * n.n_pops + b]);
      int64_t Nb = n.pop_off[b + 1] - n.pop_off[b];
      for (long long q = 0; q < K; ++q, ++m) {
        Word4 w = philox((uint64_t)j, (uint64_t)(m >> 2), 0, TAG_SRC, c.seed, 0);
        uint64_t u = upper32(w.v[m & 3]);
        int64_t src = n.pop_off[b] + (int64_t)((u * (uint64_t)Nb) >> 32);
        Syn s; s.src = src; s.tgt = (int32_t)j; s.slot = (int32_t)m;
        if (!draw_weight_delay(n, (uint64_t)j, (uint64_t)m, a, b, &s.wq, &s.d)) ok = false;
        per_target[j].push_back(s);
      }
    }
  }
  if (!ok) return false;
  std::vector<Syn> all;
  for (auto& v : per_target) all.insert(all.end(), v.begin(), v.end());
  std::stable_sort(all.begin(), all.end(), [](const Syn& x, const Syn& y) {
    if (x.src != y.src) return x.src < y.src;
    if (x.tgt != y.tgt) return x.tgt < y.tgt;
    return x.slot < y.slot;
  });
  n.row_ptr.assign((size_t)n.N + 1, 0);
  for (auto& s : all) n.row_ptr[s.src + 1]++;
  for (int64_t i = 0; i < n.N; ++i) n.row_ptr[i + 1] += n.row_ptr[i];
  n.tgt.resize(all.size()); n.wq.resize(all.size()); n.dly.resize(all.size());
  for (size_t k = 0; k < all.size(); ++k) { n.tgt[k] = all[k].tgt; n.wq[k] = all[k].wq; n.dly[k] = all[k].d; }
  return true;
}

// Pairwise Bernoulli: source i connects to target j (autapses allowed, no
// multapses) iff a 32-bit uniform keyed by (i, j) is below floor(p * 2^32).
void bernoulli_row(const Net& n, int64_t i, std::vector<int32_t>& tg) {
  const orc_cfg& c = n.cfg;
  int b = n.pop_of[i];
  tg.clear();
  for (int64_t j = 0; j < n.N; ++j) {
    int a = n.pop_of[j];
    double p = c.conn[a * n.n_pops + b];
    uint64_t T = (uint64_t)std::floor(p * 4294967296.0);
    Word4 w = philox((uint64_t)i, (uint64_t)(j >> 2), 0, TAG_CONN, c.seed, 0);
    uint64_t u = upper32(w.v[j & 3]);
    if (u < T) tg.push_back((int32_t)j);
  }
}

bool build_bernoulli(Net& n) {
  std::vector<std::vector<int32_t>> rows((size_t)n.N);
  std::vector<std::vector<int32_t>> rw((size_t)n.N);
  std::vector<std::vector<uint8_t>> rd((size_t)n.N);
  bool ok = true;
#pragma omp parallel for schedule(dynamic, 16) reduction(&& : ok)
  for (int64_t i = 0; i < n.N; ++i) {
    bernoulli_row(n, i, rows[i]);
    int b = n.pop_of[i];
    rw[i].resize(rows[i].size()); rd[i].resize(rows[i].size());
    for (size_t k = 0; k < rows[i].size(); ++k) {
      int64_t j = rows[i][k];
      if (!draw_weight_delay(n, (uint64_t)i, (uint64_t)j, n.pop_of[j], b, &rw[i][k], &rd[i][k])) ok = false;
    }
  }
  if (!ok) return false;
  n.row_ptr.assign((size_t)n.N + 1, 0);
  for (int64_t i = 0; i < n.N; ++i) n.row_ptr[i + 1] = n.row_ptr[i] + (int64_t)rows[i].size();
  int64_t M = n.row_ptr[n.N];
  n.tgt.resize((size_t)M); n.wq.resize((size_t)M); n.dly.resize((size_t)M);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < n.N; ++i) {
    int64_t o = n.row_ptr[i];
    for (size_t k = 0; k < rows[i].size(); ++k) { n.tgt[o + k] = rows[i][k]; n.wq[o + k] = rw[i][k]; n.dly[o + k] = rd[i][k]; }
    std::vector<int32_t>().swap(rows[i]); std::vector<int32_t>().swap(rw[i]); std::vector<uint8_t>().swap(rd[i]);
  }
  return true;
}

void init_state(Net& n) {
  const orc_cfg& c = n.cfg;
  n.y.assign((size_t)n.N, 0.0);
  n.I.assign((size_t)n.N, 0.0);
  n.r.assign((size_t)n.N, 0);
  for (int64_t i = 0; i < n.N; ++i) {
    Word4 w = philox((uint64_t)(i >> 2), 0, 0, TAG_V0, c.seed, 0);
    double u = unit53(w.v[i & 3]);
    n.y[i] = (c.v0_hi - c.v0_lo) * u + (c.v0_lo - c.e_l);
  }
  n.D = c.d_max_steps + 1;
  n.ring.assign((size_t)n.D, std::vector<int64_t>((size_t)n.N, 0));
  n.step = 0;
  n.raster_step.clear(); n.raster_id.clear();
  n.spikes_per_pop.assign((size_t)n.n_pops, 0);
  n.events = 0;
}

// Number of external Poisson inputs of neuron i in step `step`: the smallest k
// with u < T[k], u the upper 32 bits of word i&3 of the block keyed by
// (step, i>>2).
int poisson_count(const Net& n, int64_t step, int64_t i) {
  Word4 w = philox((uint64_t)step, (uint64_t)(i >> 2), 0, TAG_DRIVE, n.cfg.seed, 0);
  uint64_t u = upper32(w.v[i & 3]);
  const uint64_t* T = &n.table[(size_t)n.pop_of[i] * 64];
  int k = 0;
  while (u >= T[k]) ++k;
  return k;
}

// One step of the simulation cycle: update every neuron (reading and clearing
// this step's input slot), then deliver every spike of the step through its
// source's synapses into the slot `delay` steps ahead.
void run_one_step(Net& n, std::vector<int64_t>* x_record, std::vector<uint8_t>* type_record,
                  std::vector<double>* y_record, int64_t rec0 = 0) {
  const int64_t s = n.step;
  const int64_t row = s - rec0;                   // record row of this step
  std::vector<int64_t>& slot = n.ring[(size_t)(s % n.D)];
  std::vector<uint8_t> spiked((size_t)n.N, 0);
  const double Ie = n.cfg.i_e;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n.N; ++i) {
    int64_t x_int = slot[i] + (int64_t)poisson_count(n, s, i) * n.jext_q;
    slot[i] = 0;
    double x = (double)x_int * 0x1p-16;
    bool is_free = (n.r[i] == 0);
    if (is_free) {
      double yn = n.P22 * n.y[i] + n.P21 * n.I[i];
      if (Ie != 0.0) yn = yn + n.P20 * Ie;
      n.y[i] = yn;
    } else {
      n.r[i] = n.r[i] - 1;
    }
    n.I[i] = n.P11 * n.I[i] + x;
    uint8_t type = is_free ? 0 : 2;               // 0 free, 1 spike, 2 refractory
    if (is_free && n.y[i] >= n.theta) {
      spiked[i] = 1;
      n.y[i] = n.y_reset;
      n.r[i] = n.ref_steps;
      type = 1;
    }
    if (x_record) (*x_record)[(size_t)row * n.N + i] = x_int;
    if (type_record) (*type_record)[(size_t)row * n.N + i] = type;
    if (y_record) (*y_record)[(size_t)(row + 1) * n.N + i] = n.y[i];
  }
  for (int64_t i = 0; i < n.N; ++i) {
    if (!spiked[i]) continue;
    n.raster_step.push_back((int32_t)s);
    n.raster_id.push_back((int32_t)i);
    n.spikes_per_pop[n.pop_of[i]]++;
    for (int64_t k = n.row_ptr[i]; k < n.row_ptr[i + 1]; ++k) {
      n.ring[(size_t)((s + n.dly[k]) % n.D)][n.tgt[k]] += n.wq[k];
    }
    n.events += n.row_ptr[i + 1] - n.row_ptr[i];
  }
  n.step = s + 1;
}

bool setup_sizes(Net& n) {
  const orc_cfg& c = n.cfg;
  if (c.n_pops < 1 || c.n_pops > ORC_MAXPOP) return false;
  n.n_pops = c.n_pops;
  n.pop_off.assign((size_t)n.n_pops + 1, 0);
  for (int p = 0; p < n.n_pops; ++p) n.pop_off[p + 1] = n.pop_off[p] + scaled_size(c.scale, c.pop_size[p]);
  n.N = n.pop_off[n.n_pops];
  n.pop_of.resize((size_t)n.N);
  for (int p = 0; p < n.n_pops; ++p)
    for (int64_t i = n.pop_off[p]; i < n.pop_off[p + 1]; ++i) n.pop_of[i] = p;
  make_propagators(n);
  make_table(n);
  n.jext_q = std::llrint(c.w_ext * 65536.0);
  n.ref_steps = (int)std::llrint(c.t_ref / c.h);
  n.theta = c.v_th - c.e_l;
  n.y_reset = c.v_reset - c.e_l;
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C interface for the test harness (ctypes)
// ---------------------------------------------------------------------------
extern "C" {

void orc_set_threads(int n) { omp_set_num_threads(n); }

void orc_philox(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
  Word4 w = philox(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
  for (int i = 0; i < 4; ++i) out[i] = w.v[i];
}

void orc_philox_many(int64_t n, const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) orc_philox(ctr + 4 * k, key + 2 * k, out + 4 * k);
}

double orc_box_muller(const uint64_t* w4) {
  Word4 w; for (int i = 0; i < 4; ++i) w.v[i] = w4[i];
  return box_muller(w);
}

// Scale of batched instance b: 0.05 + 0.20 * u53 of word 0 of the block keyed
// by (b, 0, 0, SCALE) under key (1, 0).
double orc_instance_scale(int64_t b) {
  Word4 w = philox((uint64_t)b, 0, 0, TAG_SCALE, 1, 0);
  return 0.05 + 0.20 * unit53(w.v[0]);
}

void* orc_build(const orc_cfg* cfg) {
  Net* n = new Net();
  n->cfg = *cfg;
  if (!setup_sizes(*n)) { delete n; return nullptr; }
  bool ok = (cfg->rule == 0) ? build_fixed_indegree(*n) : build_bernoulli(*n);
  if (!ok) { delete n; return nullptr; }
  init_state(*n);
  return n;
}

// Builds sizes, propagators and tables only (no synapses, no state).
void* orc_build_params(const orc_cfg* cfg) {
  Net* n = new Net();
  n->cfg = *cfg;
  if (!setup_sizes(*n)) { delete n; return nullptr; }
  return n;
}

void orc_free(void* h) { delete (Net*)h; }

void orc_sizes(void* h, int64_t* N, int64_t* M) {
  Net* n = (Net*)h; *N = n->N; *M = n->row_ptr.empty() ? 0 : n->row_ptr[n->N];
}

void orc_pop_offsets(void* h, int64_t* off) {
  Net* n = (Net*)h; for (int p = 0; p <= n->n_pops; ++p) off[p] = n->pop_off[p];
}

void orc_synapses(void* h, int64_t* row_ptr, int32_t* tgt, int32_t* wq, uint8_t* dly) {
  Net* n = (Net*)h;
  std::memcpy(row_ptr, n->row_ptr.data(), sizeof(int64_t) * (n->N + 1));
  size_t M = n->tgt.size();
  std::memcpy(tgt, n->tgt.data(), sizeof(int32_t) * M);
  std::memcpy(wq, n->wq.data(), sizeof(int32_t) * M);
  std::memcpy(dly, n->dly.data(), M);
}

// One Bernoulli row (targets only) without building the network; returns
// the row length, writing at most `cap` targets.
int64_t orc_bernoulli_row(void* h, int64_t i, int32_t* tgt, int64_t cap) {
  Net* n = (Net*)h;
  std::vector<int32_t> tg;
  bernoulli_row(*n, i, tg);
  for (size_t k = 0; k < tg.size() && (int64_t)k < cap; ++k) tgt[k] = tg[k];
  return (int64_t)tg.size();
}

// Weight and delay of the synapse keyed (a, b) between populations post/pre.
int orc_weight_delay(void* h, uint64_t a, uint64_t b, int post, int pre, int32_t* wq, uint8_t* d) {
  Net* n = (Net*)h;
  return draw_weight_delay(*n, a, b, post, pre, wq, d) ? 0 : -1;
}

void orc_propagators(void* h, double* p) {
  Net* n = (Net*)h; p[0] = n->P11; p[1] = n->P21; p[2] = n->P22; p[3] = n->P20;
}

void orc_tables(void* h, uint64_t* T) {
  Net* n = (Net*)h; std::memcpy(T, n->table.data(), sizeof(uint64_t) * n->table.size());
}

int64_t orc_jext_q(void* h) { return ((Net*)h)->jext_q; }

int orc_poisson_count(void* h, int64_t step, int64_t i) { return poisson_count(*(Net*)h, step, i); }

// Simulate `steps` steps; returns the wall time in seconds of the loop.
double orc_run(void* h, int64_t steps) {
  Net* n = (Net*)h;
  auto t0 = std::chrono::steady_clock::now();
  for (int64_t k = 0; k < steps; ++k) run_one_step(*n, nullptr, nullptr, nullptr);
  auto t1 = std::chrono::steady_clock::now();
  return std::chrono::duration<double>(t1 - t0).count();
}

int64_t orc_step(void* h) { return ((Net*)h)->step; }

void orc_state(void* h, double* y, double* I, int32_t* r) {
  Net* n = (Net*)h;
  std::memcpy(y, n->y.data(), sizeof(double) * n->N);
  std::memcpy(I, n->I.data(), sizeof(double) * n->N);
  std::memcpy(r, n->r.data(), sizeof(int32_t) * n->N);
}

void orc_set_state(void* h, const double* y, const double* I, const int32_t* r) {
  Net* n = (Net*)h;
  std::memcpy(n->y.data(), y, sizeof(double) * n->N);
  std::memcpy(n->I.data(), I, sizeof(double) * n->N);
  std::memcpy(n->r.data(), r, sizeof(int32_t) * n->N);
}

// Logical ring: pending[k][i] is the integer input neuron i will read at step
// (current step + k), for k in [0, depth).  Entries beyond the oracle's own
// ring depth are zero.
void orc_ring(void* h, int64_t depth, int64_t* pending) {
  Net* n = (Net*)h;
  for (int64_t k = 0; k < depth; ++k)
    for (int64_t i = 0; i < n->N; ++i)
      pending[k * n->N + i] = (k < n->D) ? n->ring[(size_t)((n->step + k) % n->D)][i] : 0;
}

// Add integer input to the logical ring (test injection of single inputs).
void orc_inject(void* h, int64_t k, int64_t i, int64_t value) {
  Net* n = (Net*)h;
  n->ring[(size_t)((n->step + k) % n->D)][i] += value;
}

int64_t orc_raster_count(void* h) { return (int64_t)((Net*)h)->raster_step.size(); }

void orc_raster(void* h, int32_t* steps, int32_t* ids) {
  Net* n = (Net*)h;
  std::memcpy(steps, n->raster_step.data(), sizeof(int32_t) * n->raster_step.size());
  std::memcpy(ids, n->raster_id.data(), sizeof(int32_t) * n->raster_id.size());
}

void orc_counters(void* h, int64_t* spikes_per_pop, int64_t* events) {
  Net* n = (Net*)h;
  for (int p = 0; p < n->n_pops; ++p) spikes_per_pop[p] = n->spikes_per_pop[p];
  *events = n->events;
}

// ---------------------------------------------------------------------------
// Adjoint of L = 1/(N*S) * sum_i sum_{n<S} (y_i(n+1) - y*)^2 over the window of
// S steps that starts at the current step n0 (n counts from n0), spikes
// frozen.  The state at n0, with the input still pending from spikes before
// n0, is the fixed initial condition: only the window's own spikes carry
// weights that the gradient sees.  Step n maps
// (y_n, I_n) -> (y_{n+1}, I_{n+1}):
//   free, no spike : y' = P22 y + P21 I,  I' = P11 I + x_n
//   spike (reset)  : y' = y_reset (constant),  I' = P11 I + x_n
//   refractory     : y' = y,  I' = P11 I + x_n
// The adjoint runs backwards with lam = Ly_{n+1} + g_n, g_n = c*(y_{n+1}-y*),
// c = 2/(N*S):  Ly_n = P22*lam | 0 | lam,  LI_n = P11*LI_{n+1} + [free]*P21*lam,
// LI_S = Ly_S = 0.  A weight w_s (pA) of a synapse from i to j with delay d
// enters x_j(t+d) for each spike (t, i) of the window, so dL/dw_s =
// sum_t LI_j(t+d+1), accumulated per synapse in decreasing t.
// grad_mode 0: double accumulation; 1: float accumulation g = f(g + f(LI)).
// ---------------------------------------------------------------------------
int orc_adjoint(void* h, int64_t S, double y_star_rel, int grad_mode, void* grad_out, double* loss_out) {
  Net* n = (Net*)h;
  const int64_t N = n->N, n0 = n->step;
  const int64_t q0 = (int64_t)n->raster_step.size();   // the window's spikes follow
  std::vector<double> yrec((size_t)(S + 1) * N);
  std::vector<uint8_t> types((size_t)S * N);
  for (int64_t i = 0; i < N; ++i) yrec[i] = n->y[i];
  for (int64_t s = 0; s < S; ++s) run_one_step(*n, nullptr, &types, &yrec, n0);
  const double c = 2.0 / ((double)N * (double)S);
  double loss = 0.0;
  for (int64_t s = 0; s < S; ++s)
    for (int64_t i = 0; i < N; ++i) { double e = yrec[(size_t)(s + 1) * N + i] - y_star_rel; loss += e * e; }
  *loss_out = loss / ((double)N * (double)S);
  std::vector<double> LI((size_t)(S + 1) * N, 0.0);
  std::vector<double> Ly((size_t)N, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    double ly = 0.0, li = 0.0;      // Ly_S, LI_S
    for (int64_t s = S - 1; s >= 0; --s) {
      double g = c * (yrec[(size_t)(s + 1) * N + i] - y_star_rel);
      double lam = ly + g;
      uint8_t t = types[(size_t)s * N + i];
      double li_new = n->P11 * li;
      if (t == 0) { li_new = li_new + n->P21 * lam; ly = n->P22 * lam; }
      else if (t == 1) { ly = 0.0; }
      else { ly = lam; }
      li = li_new;
      LI[(size_t)s * N + i] = li;
    }
    Ly[i] = ly;
  }
  const int64_t M = n->row_ptr[N];
  if (grad_mode == 0) { double* g = (double*)grad_out; for (int64_t k = 0; k < M; ++k) g[k] = 0.0; }
  else { float* g = (float*)grad_out; for (int64_t k = 0; k < M; ++k) g[k] = 0.0f; }
  // the window's spikes in decreasing step order (t counted from n0)
  for (int64_t q = (int64_t)n->raster_step.size() - 1; q >= q0; --q) {
    int64_t t = n->raster_step[q] - n0, i = n->raster_id[q];
    for (int64_t k = n->row_ptr[i]; k < n->row_ptr[i + 1]; ++k) {
      int64_t m = t + n->dly[k] + 1;
      if (m > S - 1) continue;
      double v = LI[(size_t)m * N + n->tgt[k]];
      if (grad_mode == 0) ((double*)grad_out)[k] += v;
      else { float* g = (float*)grad_out; g[k] = (float)(g[k] + (float)v); }
    }
  }
  return 0;
}

// Central difference of the same loss with respect to the weight of synapse
// k, in quad precision, spikes frozen: only target j's trajectory depends on
// w_k, so it is recomputed from its recorded integer inputs with x_j(t+d)
// shifted by +-eps pA at every arrival, inside the window, from a spike of
// the window (the window starts at the current step, as in orc_adjoint; the
// forward is run here).  Returns results in `out`.
int orc_fd(void* h, int64_t S, double y_star_rel, double eps, const int64_t* syn, int64_t count, double* out) {
  Net* n = (Net*)h;
  const int64_t N = n->N, n0 = n->step;
  const size_t q0 = n->raster_step.size();
  std::vector<int64_t> xrec((size_t)S * N);
  std::vector<uint8_t> types((size_t)S * N);
  std::vector<double> y0(n->y), I0(n->I);
  for (int64_t s = 0; s < S; ++s) run_one_step(*n, &xrec, &types, nullptr, n0);
  for (int64_t q = 0; q < count; ++q) {
    int64_t k = syn[q];
    int64_t i = (int64_t)(std::upper_bound(n->row_ptr.begin(), n->row_ptr.end(), k) - n->row_ptr.begin()) - 1;
    int64_t j = n->tgt[k];
    int64_t d = n->dly[k];
    std::vector<uint8_t> hit((size_t)S, 0);
    for (size_t z = q0; z < n->raster_step.size(); ++z)
      if (n->raster_id[z] == i) { int64_t m = n->raster_step[z] - n0 + d; if (m <= S - 1) hit[m] = 1; }
    __float128 P11 = n->P11, P21 = n->P21, P22 = n->P22, P20 = n->P20;
    __float128 Lpm[2];
    for (int sg = 0; sg < 2; ++sg) {
      __float128 e = (sg == 0) ? (__float128)eps : -(__float128)eps;
      __float128 y = y0[j], I = I0[j], L = 0;
      for (int64_t s = 0; s < S; ++s) {
        __float128 x = (__float128)xrec[(size_t)s * N + j] / (__float128)65536.0;
        if (hit[s]) x += e;
        uint8_t t = types[(size_t)s * N + j];
        if (t == 0) { y = P22 * y + P21 * I; if (n->cfg.i_e != 0.0) y += P20 * (__float128)n->cfg.i_e; }
        else if (t == 1) y = n->y_reset;
        I = P11 * I + x;
        __float128 dv = y - (__float128)y_star_rel;
        L += dv * dv;
      }
      Lpm[sg] = L;
    }
    __float128 fd = (Lpm[0] - Lpm[1]) / (2 * (__float128)eps) / ((__float128)N * (__float128)S);
    out[q] = (double)fd;
  }
  return 0;
}

// The recorded step types of neuron i over a forward of S steps from the
// current step (0 free, 1 spike, 2 refractory), its integer inputs and its
// y before and after each step: for tests.
int orc_trace(void* h, int64_t S, int64_t i, uint8_t* types_out, int64_t* x_out, double* y_out) {
  Net* n = (Net*)h;
  const int64_t N = n->N, n0 = n->step;
  std::vector<int64_t> xrec((size_t)S * N);
  std::vector<uint8_t> types((size_t)S * N);
  std::vector<double> yrec((size_t)(S + 1) * N);
  for (int64_t k = 0; k < N; ++k) yrec[k] = n->y[k];
  for (int64_t s = 0; s < S; ++s) run_one_step(*n, &xrec, &types, &yrec, n0);
  for (int64_t s = 0; s < S; ++s) { types_out[s] = types[(size_t)s * N + i]; x_out[s] = xrec[(size_t)s * N + i]; }
  for (int64_t s = 0; s <= S; ++s) y_out[s] = yrec[(size_t)s * N + i];
  return 0;
}

// ---------------------------------------------------------------------------
// Learning on the stored weights (Discussion: with every synapse's weight
// stored explicitly, plasticity and learning can act on each one).  Plain
// gradient descent with step eta: w <- w - eta * g, with w in pA (the stored
// integer times 2^-16) and g the gradient orc_adjoint returns; the result is
// stored again in units of 2^-16 pA, rounded to the nearest integer with
// ties to even.  A step that would make any weight non-finite or take it
// beyond the int32 range changes nothing and returns -1.
// ---------------------------------------------------------------------------
int orc_apply_gradient(void* h, const void* grad, int grad_mode, double eta) {
  Net* n = (Net*)h;
  const int64_t M = (int64_t)n->wq.size();
  std::vector<int32_t> next((size_t)M);
  for (int64_t k = 0; k < M; ++k) {
    double g = (grad_mode == 0) ? ((const double*)grad)[k] : (double)((const float*)grad)[k];
    double w_pA = (double)n->wq[k] / 65536.0;      // exact: a power-of-two scaling
    double w_new = w_pA - eta * g;
    double units = w_new * 65536.0;                 // exact
    if (!(std::fabs(units) <= 2147483647.0)) return -1;
    next[(size_t)k] = (int32_t)std::llrint(units);  // default rounding mode: nearest, ties to even
  }
  n->wq.swap(next);
  return 0;
}

// Back to the initial state of a freshly built network (membrane potentials
// drawn again from the same keys, currents, refractory counts and input
// buffers zero, step 0, raster and counters empty); the synapse store, with
// any weights changed since the build, is kept.
void orc_reset(void* h) { init_state(*(Net*)h); }

}  // extern "C"
