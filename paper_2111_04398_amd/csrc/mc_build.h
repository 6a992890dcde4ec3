// mc_build.h -- host-side network construction of libmc (C++/OpenMP).
#pragma once
#include <stdint.h>
#include <string>
#include <vector>

#include "mc.h"

namespace mc {

struct HostNet {
  // sizes
  int n_pops = 0;
  int n_inst = 0;
  int64_t N = 0;                         // neurons (dense global ids)
  int64_t M = 0;                         // synapses
  std::vector<int64_t> inst_off;         // [n_inst+1] dense
  std::vector<int64_t> pop_off;          // [n_inst*(n_pops+1)] dense global
  std::vector<uint64_t> inst_seed;       // [n_inst]
  std::vector<double> inst_scale;        // [n_inst]
  std::vector<uint8_t> pop_of;           // [N]
  // synapse store, canonical order
  std::vector<int64_t> row_ptr;          // [N+1]
  std::vector<int32_t> tgt;              // [M]
  std::vector<int32_t> wq;               // [M], 2^-16 pA
  std::vector<uint8_t> dly;              // [M], steps
  int max_row = 0;
  int max_delay = 0;                     // largest delay in the store (steps)
  // dynamics constants
  double P11 = 0, P21 = 0, P22 = 0, P20 = 0;
  double i_e = 0, theta = 0, y_reset = 0, e_l = 0;   // theta, y_reset relative to E_L
  int64_t jext_q = 0;
  int ref_steps = 0;
  std::vector<uint64_t> table;           // [n_pops*64]
  std::vector<double> y0;                // [N]
};

// One instance of the pairwise Bernoulli rule, as a connection builder on
// another processor sees it: source i connects to target j (local ids) iff
// the upper 32 bits of word j&3 of the Philox block keyed (i, j>>2, 0, CONN)
// are below thr[pop(j) * n_pops + pop(i)].
struct BernoulliPlan {
  int64_t N = 0;               // neurons of the instance
  int n_pops = 0;
  const int64_t* off = nullptr;    // [n_pops+1] local population offsets
  const uint8_t* pop = nullptr;    // [N] local population of every neuron
  const uint64_t* thr = nullptr;   // [n_pops*n_pops] floor(p * 2^32), [post][pre]
  uint64_t seed = 0;
  int64_t goff = 0;            // global id of the instance's first neuron
};

// One instance of the fixed in-degree rule: target j draws, for each
// presynaptic population b in order, K[pop(j) * n_pops + b] sources of b
// uniformly with replacement; its draw m (m counts all its draws) is
// off[b] + ((u * N_b) >> 32) with u the upper 32 bits of word m&3 of the
// Philox block keyed (j, m>>2, 0, SRC).
struct FixedPlan {
  int64_t N = 0;
  int n_pops = 0;
  const int64_t* off = nullptr;    // [n_pops+1] local population offsets
  const uint8_t* pop = nullptr;    // [N]
  const int64_t* K = nullptr;      // [n_pops*n_pops] draws, [post][pre]
  const int64_t* first = nullptr;  // [N+1] offset of target j's draws
  uint64_t seed = 0;
};

// Draws the connections of an instance elsewhere (the HIP device).  For the
// Bernoulli rule count() gives every source's number of targets, fill() every
// source's targets (global ids, ascending) at row_ptr_local[i] -
// row_ptr_local[0] of tgt; for the fixed in-degree rule sources() gives
// every draw's local source at first[j] + m.  All must equal the host's
// draws bit for bit.
struct ConnBuilder {
  virtual ~ConnBuilder() = default;
  virtual int count(const BernoulliPlan& plan, int64_t* counts, std::string& err) = 0;
  virtual int fill(const BernoulliPlan& plan, const int64_t* row_ptr_local, int32_t* tgt, std::string& err) = 0;
  virtual int sources(const FixedPlan& plan, int32_t* src, std::string& err) = 0;
};

// Validates the configuration and builds the whole network.  With `conn`,
// the connections of the Bernoulli rule come from it (weights and delays
// stay on the host).  Returns an mc_status; on failure `err` holds a message.
int build_host(const mc_config& cfg, HostNet& net, std::string& err, ConnBuilder* conn = nullptr);

}  // namespace mc
