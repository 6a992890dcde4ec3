// mc_adjoint.hip -- reverse-time adjoint of the membrane-potential loss with
// respect to every synaptic weight, spike pattern held fixed.
//
// Loss over a window of S steps starting at step n0:
//   L = 1/(N S) sum_i sum_{n0 <= n < n0+S} (y_i(n+1) - y*)^2 .
// With the step types frozen (free / spike / refractory), the step map
// (y, I) -> (y', I') is linear: free y' = P22 y + P21 I, spike y' = y_reset,
// refractory y' = y, and always I' = P11 I + x_n.  Its transpose runs
// backwards per neuron:
//   lam  = Ly(n+1) + c (y(n+1) - y*),  c = 2/(N S)
//   LI(n) = P11 LI(n+1) + [free] P21 lam
//   Ly(n) = P22 lam | 0 | lam            (free | spike | refractory)
// with LI = Ly = 0 after the window.  The weight w_s (pA) of a synapse i -> j
// with delay d enters x_j(t + d) for each spike of i at step t, so
// dL/dw_s = sum over those spikes of LI_j(t + d + 1) (terms with
// t + d + 1 > n0 + S - 1 vanish).  The paper's explicit per-synapse weights
// (Discussion: synaptic plasticity needs them) are what make this gradient a
// per-synapse quantity.
//
// Memory: the forward keeps (y, I, r, ring) every K steps.  Segments are then
// processed last to first.  For segment [a, a+len):
//   1. k_adj_seed      x_seg[j][i] <- pending input of step a+j from the
//                      checkpointed ring (spikes before a);
//   2. (k_replay)      the recorded spikes of steps [a, a+len-1) add their
//                      weights into x_seg (integer sums: the same inputs the
//                      forward saw);
//   3. k_adj_segment   one thread per neuron: re-runs the len steps from the
//                      checkpoint (drive + exact integration, bit-identical
//                      to the forward; the drive is redrawn only when the
//                      input comes from the replay, the forward's input
//                      record already holds it), keeps y and the step type
//                      of every step, then runs the transposed recurrence
//                      backwards over the segment, writing LI into a ring of
//                      R slots;
//   4. k_adj_verify    every recorded spike of the segment must be a spike
//                      of the recompute (and the counts must agree);
//   5. k_adj_gather    one wavefront per (source, chunk of 256 of its row): for
//                      every synapse, adds LI_tgt(t + d + 1) over the
//                      source's spikes t in [a-2, a+len-2), latest first,
//                      into grad[s] (FP64, or FP32 as g = f32(g + f32(LI))).
// Segments go latest first and each segment's spikes latest first, so every
// synapse accumulates its terms in decreasing spike time.
#pragma clang fp contract(off)

#include "mc_lif.h"

namespace mc {

constexpr int kAdjBlock = 256;

// x_seg[j][i] for j in [0, rows): the checkpointed ring's slot for step a+j
// (j < ring slots), else 0.
__global__ __launch_bounds__(kAdjBlock) void k_adj_seed(long long* xseg, const long long* ring_ckpt, long long stride,
                                                        long long a, int rows) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= stride || j >= rows) return;
  xseg[(size_t)j * stride + i] = (j < kRingSlots) ? ring_ckpt[(size_t)((a + j) & kRingMask) * stride + i] : 0;
}

__global__ __launch_bounds__(kAdjBlock) void k_adj_segment(DevNet p, AdjSeg s) {
  __shared__ uint64_t s_table[kMaxPops * kTableLen];
  __shared__ unsigned s_cnt;
  for (int k = threadIdx.x; k < p.n_pops * kTableLen; k += blockDim.x) s_table[k] = p.table[k];
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();

  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long st = p.ring_stride;
  unsigned spikes = 0;
  const unsigned pop = (i < p.n_pad) ? ((p.qpops[i >> 2] >> (8 * (i & 3))) & 0xFFu) : 0xFFu;
  if (pop != 0xFFu) {
    const uint64_t* T = s_table + pop * kTableLen;
    const uint64_t qseed = p.qseed[i >> 2];
    const uint64_t qlocal = p.qlocal[i >> 2];
    const int word = (int)(i & 3);
    // forward recompute of the segment
    double y = s.ck_y[i], I = s.ck_I[i];
    int r = s.ck_r[i];
    for (int j = 0; j < s.len; ++j) {
      const long long n = s.a + j;
      long long x_int = s.xseg[(size_t)j * st + i];
      if (!s.x_has_drive) {
        const U64x4 v = philox4x64_10((uint64_t)n, qlocal, 0, kTagDrive, qseed, 0);
        x_int += (long long)poisson_from_u32(T, hi32(pick(v, word))) * p.jext_q;
      }
      uint8_t type;
      if (lif_step(p, y, I, r, x_int, type)) ++spikes;
      s.rec_y[(size_t)j * st + i] = y;
      s.rec_t[(size_t)j * st + i] = type;
    }
    // transposed recurrence, latest step first
    double ly = s.carry_ly[i], li = s.carry_li[i], loss = 0.0;
    for (int j = s.len - 1; j >= 0; --j) {
      const double e = s.rec_y[(size_t)j * st + i] - s.ystar;
      const uint8_t type = s.rec_t[(size_t)j * st + i];
      loss = loss + e * e;
      const double g = s.c * e;
      const double lam = ly + g;
      double li_new = p.P11 * li;
      if (type == kTypeFree) {
        li_new = li_new + p.P21 * lam;
        ly = p.P22 * lam;
      } else if (type == kTypeSpike) {
        ly = 0.0;
      } else {
        ly = lam;
      }
      li = li_new;
      s.li_ring[(size_t)((s.a + j) & (s.R - 1)) * st + i] = li;
    }
    s.carry_ly[i] = ly;
    s.carry_li[i] = li;
    s.loss_part[i] = s.loss_part[i] + loss;
  }
  if (spikes) atomicAdd(&s_cnt, spikes);
  __syncthreads();
  if (threadIdx.x == 0 && s_cnt) atomicAdd(s.spike_count, (unsigned long long)s_cnt);
}

// Every recorded spike (t, i) of the segment must be a spike step of the recompute.
__global__ __launch_bounds__(kAdjBlock) void k_adj_verify(const int2* spikes, int n, const uint8_t* rec_t,
                                                          long long stride, long long a, unsigned* mismatch) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int2 sp = spikes[k];
  if (rec_t[(size_t)(sp.x - a) * stride + sp.y] != kTypeSpike) atomicAdd(mismatch, 1u);
}

constexpr int kGatherChunk = 256;   // synapses per work item (4 per lane)

// Work item it: chunk it - first[j] of source j, the j with first[j] <= it
// < first[j+1]; srcs[j] = (padded source id, first spike time in `times`,
// number of its spike times, -).
template <typename G>
__global__ __launch_bounds__(kAdjBlock) void k_adj_gather(const int4* srcs, const long long* first, int nsrc,
                                                          long long n_items, const int* times, const int64_t* row_ptr,
                                                          const int32_t* tgt, const uint8_t* dly,
                                                          const double* li_ring, long long stride, int R,
                                                          long long last_m, G* grad) {
  const int lane = threadIdx.x & 63;
  const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long it = wave; it < n_items; it += nwaves) {
    int lo = 0, hi = nsrc;
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (first[mid] <= it) lo = mid; else hi = mid; }
    const int4 w = srcs[lo];
    const long long rs = row_ptr[w.x] + (it - first[lo]) * kGatherChunk;
    const long long re = min(rs + kGatherChunk, (long long)row_ptr[w.x + 1]);
#pragma unroll
    for (int u = 0; u < kGatherChunk / 64; ++u) {
      const long long e = rs + u * 64 + lane;
      if (e >= re) break;
      const int j = tgt[e];
      const int d = dly[e];
      G acc = grad[e];
      bool hit = false;
      for (int q = 0; q < w.z; ++q) {
        const long long m = (long long)times[w.y + q] + d + 1;
        if (m > last_m) continue;
        const double v = li_ring[(size_t)(m & (R - 1)) * stride + j];
        acc = (G)(acc + (G)v);
        hit = true;
      }
      if (hit) grad[e] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
hipError_t launch_adj_seed(long long* xseg, const long long* ring_ckpt, long long stride, long long a, int rows,
                           hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  const dim3 grid((unsigned)((stride + kAdjBlock - 1) / kAdjBlock), (unsigned)rows);
  hipLaunchKernelGGL(k_adj_seed, grid, dim3(kAdjBlock), 0, s, xseg, ring_ckpt, stride, a, rows);
  return hipGetLastError();
}

hipError_t launch_adj_segment(const DevNet& p, const AdjSeg& a, hipStream_t s) {
  const unsigned grid = (unsigned)((p.n_pad + kAdjBlock - 1) / kAdjBlock);
  hipLaunchKernelGGL(k_adj_segment, dim3(grid), dim3(kAdjBlock), 0, s, p, a);
  return hipGetLastError();
}

hipError_t launch_adj_verify(const int2* spikes, int n, const uint8_t* rec_t, long long stride, long long a,
                             unsigned* mismatch, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adj_verify, dim3((unsigned)((n + kAdjBlock - 1) / kAdjBlock)), dim3(kAdjBlock), 0, s, spikes,
                     n, rec_t, stride, a, mismatch);
  return hipGetLastError();
}

hipError_t launch_adj_gather(const int4* srcs, const long long* first, int nsrc, long long n_items, const int* times,
                             const int64_t* row_ptr, const int32_t* tgt, const uint8_t* dly, const double* li_ring,
                             long long stride, int R, long long last_m, void* grad, bool fp32, int grid, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_adj_gather<float>, dim3(grid), dim3(kAdjBlock), 0, s, srcs, first, nsrc, n_items, times,
                       row_ptr, tgt, dly, li_ring, stride, R, last_m, (float*)grad);
  else
    hipLaunchKernelGGL(k_adj_gather<double>, dim3(grid), dim3(kAdjBlock), 0, s, srcs, first, nsrc, n_items, times,
                       row_ptr, tgt, dly, li_ring, stride, R, last_m, (double*)grad);
  return hipGetLastError();
}

}  // namespace mc
