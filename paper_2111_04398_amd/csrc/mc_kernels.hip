// mc_kernels.hip -- HIP kernels of the simulation cycle for gfx950.
//
// Step n of the cycle (Fig. 1 caption of the paper: "update" integrates the
// state of the neurons, "deliver" distributes spike events to the targets):
//   drive   : Poisson count k_i(n) by inverse CDF of the upper 32 bits of
//             a Philox4x64-10 word keyed (n, local quad, 0, DRIVE);
//   update  : x = (ring[n][i] + k_i(n) J_q) 2^-16 pA, ring slot cleared;
//             free neurons y <- P22 y + P21 I (+ P20 I_e), refractory ones
//             count down; I <- P11 I + x; spike iff free and y >= theta,
//             then y <- y_reset, r <- t_ref/h   (exact integration, FP64,
//             no contraction);
//   compact : spike flags -> dense ascending id list per workgroup with
//             wavefront ballots and prefix sums, appended to the raster;
//   deliver : every synapse s of every spiking row adds w_q[s] to
//             ring[(n + d_s) mod 128][tgt_s] with an int64 atomic -- integer
//             sums, so the result does not depend on the order.
// Kernels are launched one per step and replayed from a HIP graph; the
// kernel boundary is the device-wide barrier between the delivery of step
// n and the update of step n+1 (the smallest delay is one step).
#pragma clang fp contract(off)

#include "mc_lif.h"

namespace mc {

constexpr int kMaxBlock = 1024;
constexpr int kMaxWaves = kMaxBlock / 64;
constexpr int kMaxQuadsPerWg = 256;             // quads updated by one workgroup of k_step

// ---------------------------------------------------------------------------
// Shared pieces
// ---------------------------------------------------------------------------

// Loads the Poisson tables of all populations into LDS.
__device__ __forceinline__ void load_tables(const DevNet& p, uint64_t* s_table) {
  for (int k = threadIdx.x; k < p.n_pops * kTableLen; k += blockDim.x) s_table[k] = p.table[k];
}

// Exclusive prefix of per-lane counts c in [0, 7] across a wavefront from
// three ballots over the bit planes of c.  Returns the lane's prefix; *total
// receives the wave total.
__device__ __forceinline__ int wave_prefix_small(int c, int* total) {
  const unsigned lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint64_t b0 = __ballot(c & 1), b1 = __ballot(c & 2), b2 = __ballot(c & 4);
  *total = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
  return __popcll(b0 & below) + 2 * __popcll(b1 & below) + 4 * __popcll(b2 & below);
}

// ---------------------------------------------------------------------------
// One step: update + compaction + owner delivery.  Workgroup g updates the
// quads [g*qpw, (g+1)*qpw) (one quad per thread), compacts its spikes into
// an ascending list in LDS, appends them to its private raster segment and
// walks their synapse rows with all of its threads.
// ---------------------------------------------------------------------------
template <bool kOwnerLists>
__global__ __launch_bounds__(kMaxBlock) void k_step(DevNet p, int offset, int qpw, int wave_rows) {
  __shared__ uint64_t s_table[kMaxPops * kTableLen];
  __shared__ int s_wcnt[kMaxWaves];
  __shared__ int s_spk[4 * kMaxQuadsPerWg];
  __shared__ long long s_rs[4 * kMaxQuadsPerWg];
  __shared__ unsigned long long s_events;

  const long long n = *p.step_base + offset;
  load_tables(p, s_table);
  __syncthreads();

  const int tid = threadIdx.x;
  const long long q = (long long)blockIdx.x * qpw + tid;
  unsigned mask = 0;
  if (tid < qpw && q < p.n_quads) {
    const uint32_t pops = p.qpops[q];
    const U64x4 v = philox4x64_10((uint64_t)n, (uint64_t)p.qlocal[q], 0, kTagDrive, p.qseed[q], 0);
    long long* slot = p.ring + (size_t)(n & kRingMask) * p.ring_stride + 4 * q;
    const longlong2 s01 = *reinterpret_cast<const longlong2*>(slot);
    const longlong2 s23 = *reinterpret_cast<const longlong2*>(slot + 2);
    *reinterpret_cast<longlong2*>(slot) = make_longlong2(0, 0);
    *reinterpret_cast<longlong2*>(slot + 2) = make_longlong2(0, 0);
    const long long sl[4] = {s01.x, s01.y, s23.x, s23.y};
    double* yq = p.y + 4 * q;
    double* Iq = p.I + 4 * q;
    int* rq = p.r + 4 * q;
    const double2 ya = *reinterpret_cast<const double2*>(yq), yb = *reinterpret_cast<const double2*>(yq + 2);
    const double2 ia = *reinterpret_cast<const double2*>(Iq), ib = *reinterpret_cast<const double2*>(Iq + 2);
    const int4 r4 = *reinterpret_cast<const int4*>(rq);
    if (p.ck_y) {                        // adjoint forward: checkpoint before the update
      const int k = (int)(n - p.ck_step0), every = (int)p.ck_every;   // windows hold at most 1e6 steps
      if (k >= 0 && k % every == 0 && k / every < p.ck_count) {
        const size_t at = (size_t)(k / every) * p.ring_stride + 4 * q;
        *reinterpret_cast<double2*>(p.ck_y + at) = ya;
        *reinterpret_cast<double2*>(p.ck_y + at + 2) = yb;
        *reinterpret_cast<double2*>(p.ck_I + at) = ia;
        *reinterpret_cast<double2*>(p.ck_I + at + 2) = ib;
        *reinterpret_cast<int4*>(p.ck_r + at) = r4;
      }
    }
    double y[4] = {ya.x, ya.y, yb.x, yb.y};
    double I[4] = {ia.x, ia.y, ib.x, ib.y};
    int r[4] = {r4.x, r4.y, r4.z, r4.w};
    uint8_t type[4];
    long long xin[4] = {sl[0], sl[1], sl[2], sl[3]};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const unsigned pop = (pops >> (8 * k)) & 0xFFu;
      if (pop == 0xFFu) continue;  // padding neuron: never updated, never spikes
      const int cnt = poisson_from_u32(s_table + pop * kTableLen, hi32(pick(v, k)));
      xin[k] = sl[k] + (long long)cnt * p.jext_q;
      if (lif_step(p, y[k], I[k], r[k], xin[k], type[k])) mask |= 1u << k;
    }
    if (p.xrec && n - p.xrec_step0 >= 0 && n - p.xrec_step0 < p.xrec_steps) {
      long long* xr = p.xrec + (size_t)(n - p.xrec_step0) * p.ring_stride + 4 * q;
      *reinterpret_cast<longlong2*>(xr) = make_longlong2(xin[0], xin[1]);
      *reinterpret_cast<longlong2*>(xr + 2) = make_longlong2(xin[2], xin[3]);
    }
    *reinterpret_cast<double2*>(yq) = make_double2(y[0], y[1]);
    *reinterpret_cast<double2*>(yq + 2) = make_double2(y[2], y[3]);
    *reinterpret_cast<double2*>(Iq) = make_double2(I[0], I[1]);
    *reinterpret_cast<double2*>(Iq + 2) = make_double2(I[2], I[3]);
    *reinterpret_cast<int4*>(rq) = make_int4(r[0], r[1], r[2], r[3]);
  }

  // compaction: ascending ids (thread order = quad order, bit order = id order)
  int wtotal;
  const int c = __popc(mask);
  const int pre = wave_prefix_small(c, &wtotal);
  const int wave = tid >> 6;
  if ((tid & 63) == 0) s_wcnt[wave] = wtotal;
  if (tid == 0) s_events = 0;
  __syncthreads();
  int woff = 0, total = 0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) { const int t = s_wcnt[w]; woff += (w < wave) ? t : 0; total += t; }
  if (mask) {
    int pos = woff + pre;
    for (int k = 0; k < 4; ++k)
      if (mask & (1u << k)) s_spk[pos++] = (int)(4 * q + k);
  }
  __syncthreads();
  if (total == 0) return;

  // row bounds, raster append, counters
  for (int s = tid; s < total; s += blockDim.x) {
    const int i = s_spk[s];
    const long long rs = p.row_ptr[i], re = p.row_ptr[i + 1];
    s_rs[s] = rs;
    atomicAdd(&s_events, (unsigned long long)(re - rs));
  }
  const long long rbase = p.raster_cnt[blockIdx.x];
  const bool fits = rbase + total <= p.raster_cap;
  for (int s = tid; s < total && fits; s += blockDim.x)
    p.raster[(size_t)blockIdx.x * p.raster_cap + rbase + s] = make_int2((int)n, s_spk[s]);
  __syncthreads();
  if (tid == 0) {
    if (fits) p.raster_cnt[blockIdx.x] = rbase + total;
    else atomicOr(p.overflow, 1u);
    p.wg_events[blockIdx.x] += s_events;
    for (int s = 0; s < total; ++s) {
      const int i = s_spk[s];
      const unsigned pop = (p.qpops[i >> 2] >> (8 * (i & 3))) & 0xFFu;
      p.wg_spikes[(size_t)blockIdx.x * p.n_pops + pop] += 1ull;
    }
  }

  if (kOwnerLists) {
    // target-owner scheme: the spikes go to their instance's list of this
    // step; the owner kernel delivers them
    const int par = (int)(n & 1);
    for (int s = tid; s < total; s += blockDim.x) {
      const int i = s_spk[s];
      const int b = p.qinst[i >> 2];
      const int pos = atomicAdd(&p.icnt[par * p.n_inst + b], 1);
      p.ilist[(size_t)par * p.n_pad + p.inst_base[b] + pos] = i;
    }
    return;
  }

  // owner delivery: all threads walk each spiking row in turn, or (wave_rows)
  // every wavefront walks whole rows, the spikes dealt round robin
  const long long nn = n;
  const int rstep = wave_rows ? (int)(blockDim.x >> 6) : 1;
  for (int s = wave_rows ? (tid >> 6) : 0; s < total; s += rstep) {
    const long long rs = s_rs[s];
    const long long re = p.row_ptr[s_spk[s] + 1];
    long long e = rs + (wave_rows ? (tid & 63) : tid);
    const int stride = wave_rows ? 64 : blockDim.x;
    for (; e + 3 * stride < re; e += 4 * stride) {
      int t[4], w[4], d[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { t[u] = p.tgt[e + u * stride]; w[u] = p.wq[e + u * stride]; d[u] = p.dly[e + u * stride]; }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        atomicAdd(reinterpret_cast<unsigned long long*>(p.ring + (size_t)((nn + d[u]) & kRingMask) * p.ring_stride + t[u]),
                  (unsigned long long)(long long)w[u]);
    }
    for (; e < re; e += stride) {
      const int t = p.tgt[e], w = p.wq[e], d = p.dly[e];
      atomicAdd(reinterpret_cast<unsigned long long*>(p.ring + (size_t)((nn + d) & kRingMask) * p.ring_stride + t),
                (unsigned long long)(long long)w);
    }
  }
}

__global__ void k_advance(long long* step_base, int steps) { *step_base += steps; }

// Adds a value to one ring entry (host-requested input injection).
__global__ void k_inject(long long* ring, long long idx, long long value) { ring[idx] += value; }

// New weights of every synapse in units of 2^-16 pA, rounded to nearest
// even.  kWeightsSet: the real weights w_pA[k]; kWeightsStepF64/F32: one
// gradient step w_q[k] 2^-16 - eta g[k] (g double or float), evaluated as
// fl(w_q 2^-16 - fl(eta g)) (the first product is exact).  check: only test
// that every new weight is finite and fits int32 (*bad = 1 if not), so that a
// rejected update leaves the store untouched; else write them.
enum { kWeightsSet = 0, kWeightsStepF64 = 1, kWeightsStepF32 = 2 };
__global__ void k_weights(int32_t* wq, const void* src, int mode, double eta, long long M, unsigned* bad, int check) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < M; k += (long long)gridDim.x * blockDim.x) {
    double w;
    if (mode == kWeightsSet) {
      w = static_cast<const double*>(src)[k];
    } else {
      const double g = (mode == kWeightsStepF64) ? static_cast<const double*>(src)[k]
                                                 : (double)static_cast<const float*>(src)[k];
      w = (double)wq[k] * 0x1p-16 - eta * g;
    }
    const double ws = w * 65536.0;
    if (check) {
      if (!(fabs(ws) <= 2147483647.0)) atomicOr(bad, 1u);
    } else {
      wq[k] = (int32_t)__double2ll_rn(ws);
    }
  }
}

// Packs the used prefixes of the per-workgroup raster segments (capacity
// `cap` entries each) into one contiguous array: workgroup g's entries go to
// out[off[g] .. off[g+1]).  One workgroup per segment.
__global__ void k_raster_pack(const int2* raster, long long cap, const long long* off, int2* out) {
  const int g = blockIdx.x;
  const long long b = off[g], c = off[g + 1] - b;
  const int2* src = raster + (size_t)g * cap;
  for (long long k = threadIdx.x; k < c; k += blockDim.x) out[b + k] = src[k];
}

}  // namespace mc

// ---------------------------------------------------------------------------
// Host-side launch wrappers (called from the C interface)
// ---------------------------------------------------------------------------
namespace mc {

hipError_t launch_step(const DevNet& p, int offset, int qpw, int n_wg, int block, int wave_rows, hipStream_t s) {
  hipLaunchKernelGGL(k_step<false>, dim3(n_wg), dim3(block), 0, s, p, offset, qpw, wave_rows);
  return hipGetLastError();
}

hipError_t launch_step_lists(const DevNet& p, int offset, int qpw, int n_wg, int block, hipStream_t s) {
  hipLaunchKernelGGL(k_step<true>, dim3(n_wg), dim3(block), 0, s, p, offset, qpw, 0);
  return hipGetLastError();
}

hipError_t launch_advance(long long* step_base, int steps, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, s, step_base, steps);
  return hipGetLastError();
}

hipError_t launch_inject(long long* ring, long long idx, long long value, hipStream_t s) {
  hipLaunchKernelGGL(k_inject, dim3(1), dim3(1), 0, s, ring, idx, value);
  return hipGetLastError();
}

hipError_t launch_raster_pack(const int2* raster, long long cap, const long long* off, int n_seg, int2* out,
                              hipStream_t s) {
  if (n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_pack, dim3((unsigned)n_seg), dim3(256), 0, s, raster, cap, off, out);
  return hipGetLastError();
}

hipError_t launch_weights(int32_t* wq, const void* src, int mode, double eta, long long M, unsigned* bad, bool check,
                          hipStream_t s) {
  if (M == 0) return hipSuccess;
  long long blocks = (M + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_weights, dim3((unsigned)blocks), dim3(256), 0, s, wq, src, mode, eta, M, bad, check ? 1 : 0);
  return hipGetLastError();
}

}  // namespace mc
