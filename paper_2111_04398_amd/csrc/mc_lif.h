// mc_lif.h -- the per-neuron arithmetic shared by the step kernel and the
// adjoint's segment recompute: Poisson count by table inversion and one
// exact-integration step of iaf_psc_exp (Methods: neuron model, h = 0.1 ms).
// Including files compile with FP contraction off, so both evaluate
// fl(fl(P22 y) + fl(P21 I)) and fl(fl(P11 I) + x) exactly as written.
#pragma once
#include "mc_device.h"

namespace mc {

// Inverse CDF: smallest k with u < T[k] (T[63] = 2^32 > u ends the search).
__device__ __forceinline__ int poisson_from_u32(const uint64_t* T, uint32_t u) {
  int k = 0;
  while ((uint64_t)u >= T[k]) ++k;
  return k;
}

// Step types recorded for the adjoint.
constexpr uint8_t kTypeFree = 0, kTypeSpike = 1, kTypeRefractory = 2, kTypePad = 3;

// One neuron's exact-integration step on the input x_int (2^-16 pA).
// Returns true on a spike; *type receives the step type.
__device__ __forceinline__ bool lif_step(const DevNet& p, double& y, double& I, int& r, long long x_int, uint8_t& type) {
  const double x = (double)x_int * 0x1p-16;
  const bool free_ = (r == 0);
  if (free_) {
    double yn = p.P22 * y + p.P21 * I;
    if (p.i_e != 0.0) yn = yn + p.P20 * p.i_e;
    y = yn;
  } else {
    r = r - 1;
  }
  I = p.P11 * I + x;
  type = free_ ? kTypeFree : kTypeRefractory;
  if (free_ && y >= p.theta) {
    y = p.y_reset;
    r = p.ref_steps;
    type = kTypeSpike;
    return true;
  }
  return false;
}

}  // namespace mc
