// mc_replay.hip -- throughput form of the delivery: the recorded spikes of
// many steps delivered in one launch, and the chip's random int64 atomic rate.
//
// In the simulation loop a step of the full microcircuit delivers only
// ~2.5e5 events, so the loop is bound by latency, not by bandwidth.  To see
// how close the delivery itself comes to the memory system's limits, the
// recorded raster of a span of steps is replayed: every synapse of every
// spike adds its weight into a ring wide enough for the whole span plus the
// largest delay, with device-scope int64 atomics (the sums are exact, so the
// result equals the sum of the in-loop deliveries whatever the order).
// Work items are fixed-size chunks of the concatenated spiking rows, one
// wavefront per chunk, so long and short rows balance.
#include "mc_device.h"

namespace mc {

constexpr int kReplayChunk = 256;     // synapses per work item (4 per lane)

// items: for spike k, chunk c -> item index first_item[k] + c
__global__ __launch_bounds__(256) void k_replay(const int2* spikes, const long long* first_item, int n_spikes,
                                                long long n_items, const int64_t* row_ptr, const int32_t* tgt,
                                                const int32_t* wq, const uint8_t* dly, long long* ring,
                                                long long stride, long long step0) {
  const int lane = threadIdx.x & 63;
  const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long item = wave; item < n_items; item += nwaves) {
    int lo = 0, hi = n_spikes;             // spike k: first_item[k] <= item < first_item[k+1]
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (first_item[mid] <= item) lo = mid; else hi = mid; }
    const int2 sp = spikes[lo];
    const long long rs = row_ptr[sp.y] + (item - first_item[lo]) * kReplayChunk;
    const long long re = min(rs + kReplayChunk, (long long)row_ptr[sp.y + 1]);
    const long long srel = sp.x - step0;
    int t[4], w[4], d[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long e = rs + u * 64 + lane;
      d[u] = 0;
      if (e < re) { t[u] = tgt[e]; w[u] = wq[e]; d[u] = dly[e]; }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (d[u]) atomicAdd(reinterpret_cast<unsigned long long*>(ring + (size_t)(srel + d[u]) * stride + t[u]),
                          (unsigned long long)(long long)w[u]);
  }
}

// Random int64 atomics into a table of `n` entries: the achievable rate of
// the memory-side atomic units for the delivery's access pattern.
__global__ __launch_bounds__(256) void k_atomic_rate(unsigned long long* table, long long n, long long per_thread,
                                                     unsigned seed) {
  const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  unsigned long long x = (unsigned long long)tid * 0x9E3779B97F4A7C15ull + seed;
  for (long long k = 0; k < per_thread; ++k) {
    x ^= x << 13; x ^= x >> 7; x ^= x << 17;
    atomicAdd(&table[(x >> 11) % (unsigned long long)n], 1ull);
  }
}

hipError_t launch_replay(const int2* spikes, const long long* first_item, int n_spikes, long long n_items,
                         const int64_t* row_ptr, const int32_t* tgt, const int32_t* wq, const uint8_t* dly,
                         long long* ring, long long stride, long long step0, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_replay, dim3(grid), dim3(256), 0, s, spikes, first_item, n_spikes, n_items, row_ptr, tgt, wq,
                     dly, ring, stride, step0);
  return hipGetLastError();
}

hipError_t launch_atomic_rate(unsigned long long* table, long long n, long long per_thread, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_atomic_rate, dim3(grid), dim3(256), 0, s, table, n, per_thread, 12345u);
  return hipGetLastError();
}

}  // namespace mc
