// mc_owner.hip -- target-owner delivery, one kernel per step.
//
// The update kernel of step n (k_step in list mode) appends every spike to
// the spike list of its instance.  Then this kernel delivers them: block k
// owns a range of targets of one instance and walks, for every spike of that
// instance, only the part of the source row that lands in its range (rows are
// sorted by target; blk2 holds the part's bounds).  The events are combined
// in an LDS hash table keyed by (delay, target), so that every ring entry the
// block touches is added to by exactly one thread with a plain load and
// store: no device atomics, whose memory-side rate (~2e10/s on this chip)
// bounds the source-owner delivery of k_step.  The ring entries of a block's
// targets belong to that block alone, and the update kernel of step n+1
// starts only after this kernel ends, so the plain read-modify-writes cannot
// race.  Integer sums: the result does not depend on the order of events.
#include <algorithm>

#include "mc_device.h"

namespace mc {

namespace {

constexpr int kHashBits = 10;
constexpr int kHash = 1 << kHashBits;   // table slots; a round inserts at most kHash entries
constexpr int kEmpty = -1;

__device__ __forceinline__ int hash_slot(int key) {
  return (int)(((unsigned)key * 2654435761u) >> (32 - kHashBits));
}

}  // namespace

__global__ __launch_bounds__(kOwnerBlock) void k_owner(DevNet p, OwnerArgs a, int offset) {
  __shared__ int s_key[kHash];
  __shared__ long long s_val[kHash];
  __shared__ int s_pre[kOwnerBlock + 1];      // exclusive prefix of the sub-row lengths of a chunk of spikes
  __shared__ long long s_lo[kOwnerBlock];
  __shared__ int s_wsum[kOwnerBlock / 64];

  const int tid = threadIdx.x;
  const int k = blockIdx.x;
  const long long n = *p.step_base + offset;
  const int par = (int)(n & 1);
  const int b = a.binst[k];
  const int lb = a.blb[k];
  const int t0 = a.bt0[k];
  const int bmax = a.bmax;
  // this block's list of step n; the first block of the instance empties the
  // list of step n+1 (its last reader was the owner kernel of step n-1; the
  // chunk's first step finds both emptied by k_zero_lists)
  const int cnt = p.icnt[par * p.n_inst + b];
  if (lb == 0 && tid == 0) p.icnt[(par ^ 1) * p.n_inst + b] = 0;
  const int* list = p.ilist + (size_t)par * p.n_pad + p.inst_base[b];
  for (int x = tid; x < kHash; x += kOwnerBlock) { s_key[x] = kEmpty; s_val[x] = 0; }

  for (int c0 = 0; c0 < cnt; c0 += kOwnerBlock) {
    // sub-row bounds of this chunk of spikes, one per thread
    int len = 0;
    long long lo = 0;
    if (c0 + tid < cnt) {
      const int i = list[c0 + tid];
      const long long rs = p.row_ptr[i];
      const int64_t o = a.boff[i] + lb;
      lo = rs + a.blk2[o];
      len = a.blk2[o + 1] - a.blk2[o];
    }
    // block-wide exclusive scan of len
    int x = len;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    __syncthreads();                          // previous chunk's readers of s_pre / s_lo are done
    if (lane == 63) s_wsum[wave] = x;
    __syncthreads();
    int woff = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kOwnerBlock / 64; ++w) { const int t = s_wsum[w]; woff += (w < wave) ? t : 0; total += t; }
    s_pre[tid] = woff + x - len;
    s_lo[tid] = lo;
    if (tid == 0) s_pre[kOwnerBlock] = total;
    __syncthreads();
    const int nsp = min(kOwnerBlock, cnt - c0);
    // rounds of at most kHash entries: the table never fills
    for (int r0 = 0; r0 < total; r0 += kHash) {
      const int r1 = min(total, r0 + kHash);
      for (int f = r0 + tid; f < r1; f += kOwnerBlock) {
        int lo_j = 0, hi_j = nsp;               // spike j: s_pre[j] <= f < s_pre[j+1]
        while (hi_j - lo_j > 1) { const int mid = (lo_j + hi_j) >> 1; if (s_pre[mid] <= f) lo_j = mid; else hi_j = mid; }
        const long long e = s_lo[lo_j] + (f - s_pre[lo_j]);
        const int t = p.tgt[e];
        const int w = p.wq[e];
        const int d = p.dly[e];
        const int key = d * bmax + (t - t0);
        int h = hash_slot(key);
        while (true) {
          const int old = atomicCAS(&s_key[h], kEmpty, key);
          if (old == kEmpty || old == key) break;
          h = (h + 1) & (kHash - 1);
        }
        atomicAdd(reinterpret_cast<unsigned long long*>(&s_val[h]), (unsigned long long)(long long)w);
      }
      __syncthreads();
      // flush: one thread per distinct (delay, target)
      for (int xk = tid; xk < kHash; xk += kOwnerBlock) {
        const int key = s_key[xk];
        if (key == kEmpty) continue;
        const int d = key / bmax;
        const int tl = key - d * bmax;
        long long* e = p.ring + (size_t)((n + d) & kRingMask) * p.ring_stride + t0 + tl;
        *e += s_val[xk];
        s_key[xk] = kEmpty;
        s_val[xk] = 0;
      }
      __syncthreads();
    }
  }
}

// blk2[boff[i] + lb] = offset inside row i of its first synapse with target
// >= bt0[first block of its instance + lb], for lb = 0 .. blocks of the
// instance (the last one: the row length).  One workgroup per row.
__global__ __launch_bounds__(64) void k_build_blk2(const int64_t* row_ptr, const int32_t* tgt, long long n_pad,
                                                   const int64_t* boff, const int32_t* qinst,
                                                   const int* inst_first_block, const int* bt0, int32_t* blk2) {
  const long long i = blockIdx.x;
  if (i >= n_pad) return;
  const int b = qinst[i >> 2];
  const int fb = inst_first_block[b];
  const int nb = (int)(boff[i + 1] - boff[i]);   // blocks of the instance + 1
  const long long rs = row_ptr[i], re = row_ptr[i + 1];
  for (int lb = threadIdx.x; lb < nb; lb += blockDim.x) {
    const int key = bt0[fb + lb];
    long long lo = rs, hi = re;
    while (lo < hi) { const long long mid = (lo + hi) >> 1; if (tgt[mid] < key) lo = mid + 1; else hi = mid; }
    blk2[boff[i] + lb] = (int32_t)(lo - rs);
  }
}

// Empties both parities of the per-instance spike lists.  Launched at the
// start of every chunk of target-owner steps: the owner kernel of step n
// empties the lists of step n+1 only, so the lists of the last step of an
// earlier chunk (possibly followed by steps of another scheme) would remain.
__global__ void k_zero_lists(int* icnt, int n) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) icnt[k] = 0;
}

hipError_t launch_zero_lists(int* icnt, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_lists, dim3((unsigned)std::min(64, (n + 255) / 256)), dim3(256), 0, s, icnt, n);
  return hipGetLastError();
}

hipError_t launch_owner(const DevNet& p, const OwnerArgs& a, int offset, hipStream_t s) {
  if (a.n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_owner, dim3((unsigned)a.n_blocks), dim3(kOwnerBlock), 0, s, p, a, offset);
  return hipGetLastError();
}

hipError_t launch_build_blk2(const int64_t* row_ptr, const int32_t* tgt, long long n_pad, const int64_t* boff,
                             const int32_t* qinst, const int* inst_first_block, const int* bt0, int32_t* blk2,
                             hipStream_t s) {
  if (n_pad <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_build_blk2, dim3((unsigned)n_pad), dim3(64), 0, s, row_ptr, tgt, n_pad, boff, qinst,
                     inst_first_block, bt0, blk2);
  return hipGetLastError();
}

}  // namespace mc
