// mc_replay.hip -- throughput form of the delivery: the recorded spikes of
// many steps delivered in one launch; and the microbenchmarks of what the
// memory system achieves for the delivery's two costs: a streaming read
// (the synapse records) and int64 atomic adds into a slot-major ring.
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

// Streaming read of `n16` 16-byte words (grid-stride, eight loads in flight
// per lane): the achievable HBM read bandwidth.  The XOR of what a thread
// read is stored only if it equals a value the data never produce, so the
// loads cannot be dropped.
__global__ __launch_bounds__(256) void k_stream_read(const ulonglong2* src, long long n16, unsigned long long* sink) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  unsigned long long x = 0;
  long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  for (; k + 7 * stride < n16; k += 8 * stride) {
    ulonglong2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[k + u * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) x ^= v[u].x ^ v[u].y;
  }
  for (; k < n16; k += stride) { const ulonglong2 a = src[k]; x ^= a.x ^ a.y; }
  if (x == 0x5A5A5A5A5A5A5A5Aull) sink[0] = x;
}

// Slot-major int64 atomic adds into table[slot][target] (slots x stride
// entries), in work items of 256 events (4 per lane, one wavefront).  The
// addresses come from a cheap 32-bit hash and multiply-shift, so that the
// probe is bound by the atomics, not by its own arithmetic.
// pattern 0: every event at a uniformly random (slot, target);
// pattern 1: the delivery's own pattern -- an item is a chunk of one source
// row at spike step t (t advancing with the item index over the first
// slots - 101 slots): targets ascending with gaps uniform in [1, 2 gap - 1],
// each event's delay one of 1024 quantiles of the network's delay
// histogram (dq), landing in slot t + delay.
__device__ __forceinline__ unsigned hash32(unsigned x) {
  x ^= x >> 16; x *= 0x7FEB352Du;
  x ^= x >> 15; x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}
__device__ __forceinline__ unsigned scale32(unsigned h, unsigned n) { return (unsigned)(((unsigned long long)h * n) >> 32); }

__global__ __launch_bounds__(256) void k_atomic_slots(unsigned long long* table, long long slots, long long stride,
                                                      long long n_targets, long long n_items, int pattern, int gap,
                                                      const unsigned char* dq) {
  __shared__ unsigned char s_dq[1024];
  for (int k = threadIdx.x; k < 1024; k += blockDim.x) s_dq[k] = dq[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  const long long tspan = slots > 101 ? slots - 101 : 1;
  const unsigned ns = (unsigned)slots, nt = (unsigned)n_targets;
  for (long long item = wave; item < n_items; item += nwaves) {
    const unsigned h0 = hash32((unsigned)item * 0x9E3779B9u + 0x632BE5ABu);
    const long long t = item * tspan / n_items;
    unsigned tg = scale32(h0, nt);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const unsigned h = hash32(h0 ^ (unsigned)(u * 64 + lane + 1) * 0x85EBCA6Bu);
      unsigned slot, target;
      if (pattern == 0) {
        slot = scale32(h, ns);
        target = scale32(hash32(h ^ 0x5BD1E995u), nt);
      } else {
        const int g = 1 + (int)scale32(h, (unsigned)(2 * gap - 1));
        int x = g;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        target = tg + (unsigned)x;
        while (target >= nt) target -= nt;
        tg += (unsigned)__shfl(x, 63, 64);
        while (tg >= nt) tg -= nt;
        slot = (unsigned)((t + s_dq[(h >> 8) & 1023]) % slots);
      }
      atomicAdd(&table[(size_t)slot * stride + target], 1ull);
    }
  }
}

hipError_t launch_stream_read(const void* src, long long bytes, unsigned long long* sink, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(256), 0, s, (const ulonglong2*)src, bytes / 16, sink);
  return hipGetLastError();
}

hipError_t launch_atomic_slots(unsigned long long* table, long long slots, long long stride, long long n_targets,
                               long long n_items, int pattern, int gap, const unsigned char* dq, int grid,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_atomic_slots, dim3(grid), dim3(256), 0, s, table, slots, stride, n_targets, n_items, pattern,
                     gap, dq);
  return hipGetLastError();
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
