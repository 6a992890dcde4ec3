// mc_persist.hip -- persistent multi-step kernel with the near-future input
// held in LDS (target-owner delivery).
//
// Why: on gfx950 a device-scope int64 atomic is performed at the memory side
// at about 20e9 per second for the whole chip, whatever the footprint of the
// table, so a step of the full microcircuit (~2.5e5 synaptic events) cannot
// drop below ~12 us if every event is a global atomic.  Here every workgroup
// owns a contiguous block of B target neurons and keeps their pending input
// for the next D_L steps in LDS (int64, LDS atomics); it delivers, for every
// spike of the step, only the part of the source row that targets its own
// block (rows are sorted by target, so that part is contiguous and an index
// blk[i][g] gives its bounds).  Events with a delay >= D_L (rare: the delay
// distribution's tail) go to the global ring with device atomics, into
// entries only the owner reads.  The only cross-workgroup traffic per step
// is the spike list: each workgroup publishes its spikes and a tagged flag,
// and every workgroup waits for all flags of the step before delivering.
//
// Memory ordering: all cross-workgroup data (spike ids, flags, global ring
// entries touched during the launch) is written and read with device-scope
// atomic operations (coherent at the memory side on this chip), and the
// producer waits for its id stores to complete (s_waitcnt) before it stores
// the flag.  No L2 writeback/invalidate fences are needed on the step path.
// Every wait is bounded; on timeout the kernel sets an error bit and all
// workgroups leave the loop.
#pragma clang fp contract(off)

#include "mc_device.h"

namespace mc {

namespace {

constexpr int kListCap = 1024;       // spikes gathered into LDS per pass
constexpr int kFlagStride = 8;       // flags 64 bytes apart (u64 units)

__device__ __forceinline__ int poisson_inv(const uint64_t* T, uint32_t u) {
  int k = 0;
  while ((uint64_t)u >= T[k]) ++k;
  return k;
}

__device__ __forceinline__ long long ld_dev(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_dev(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_dev(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide exclusive scan of v (one value per thread); returns the
// thread's exclusive prefix, *total the block sum.  s_tmp: one int per wave.
__device__ __forceinline__ int block_exscan(int v, int* s_tmp, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  int woff = 0, tot = 0;
  for (int w = 0; w < nw; ++w) { const int t = s_tmp[w]; woff += (w < wave) ? t : 0; tot += t; }
  __syncthreads();
  *total = tot;
  return woff + x - v;
}

}  // namespace

// LDS layout (dynamic): acc[DL*B] i64 | fbits[128*BW] u32 | s_cnt[G+1] | s_list[kListCap] | s_lo/len[kListCap]...
__global__ __launch_bounds__(1024) void k_persist(DevNet p, PersistArgs a, int steps) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  __shared__ uint64_t s_table[kMaxPops * kTableLen];
  __shared__ int s_tmp[16];
  __shared__ int s_local[4 * 256];
  __shared__ int s_abort;
  __shared__ unsigned long long s_events;
  __shared__ unsigned long long s_popcnt[kMaxPops];
  long long* acc = reinterpret_cast<long long*>(s_raw);
  unsigned* fbits = reinterpret_cast<unsigned*>(acc + (size_t)a.DL * a.B);
  int* s_pre = reinterpret_cast<int*>(fbits + 128 * a.BW);        // [G+1]
  int* s_list = s_pre + (a.G + 1);                                  // [kListCap]
  int* s_len = s_list + kListCap;                                   // [kListCap]
  long long* s_lo = reinterpret_cast<long long*>(((uintptr_t)(s_len + kListCap) + 15) & ~(uintptr_t)15);  // [kListCap]

  const int g = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
  const long long j0 = (long long)g * a.B;                          // first owned target (padded id)
  const int Bg = (int)max(0LL, min((long long)a.B, p.n_pad - j0));  // owned targets (multiple of 4)
  const int qw = Bg / 4;
  const long long n0 = *p.step_base;
  const int DL = a.DL;

  for (int k = tid; k < p.n_pops * kTableLen; k += nthr) s_table[k] = p.table[k];
  for (int k = tid; k < DL * a.B; k += nthr) acc[k] = 0;
  for (int k = tid; k < 128 * a.BW; k += nthr) fbits[k] = 0;
  if (tid == 0) { s_abort = 0; s_events = 0; }
  if (tid < kMaxPops) s_popcnt[tid] = 0;
  __syncthreads();
  // take the next DL steps of pending input of my targets into LDS; mark far entries
  for (int k = tid; k < 128 * Bg; k += nthr) {
    const int m = k / Bg, jl = k - m * Bg;
    const long long step = n0 + m;
    long long* e = p.ring + (size_t)(step & kRingMask) * p.ring_stride + j0 + jl;
    if (m < DL) {
      acc[(size_t)(step % DL) * a.B + jl] =
          (long long)__hip_atomic_exchange(reinterpret_cast<unsigned long long*>(e), 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (m < 127) {
      if (ld_dev(e) != 0) atomicOr(&fbits[(step & kRingMask) * a.BW + (jl >> 5)], 1u << (jl & 31));
    }
  }
  // neuron state into registers: thread t < qw owns quad t of the block
  double y[4] = {0, 0, 0, 0}, I[4] = {0, 0, 0, 0};
  int r[4] = {0, 0, 0, 0};
  uint32_t pops = 0xFFFFFFFFu, qlocal = 0;
  uint64_t seed = 0;
  const long long q = j0 / 4 + tid;
  if (tid < qw) {
    pops = p.qpops[q]; qlocal = p.qlocal[q]; seed = p.qseed[q];
    for (int k = 0; k < 4; ++k) { y[k] = p.y[4 * q + k]; I[k] = p.I[4 * q + k]; r[k] = p.r[4 * q + k]; }
  }
  long long rcnt = p.raster_cnt[g];
  __syncthreads();

  for (int it = 0; it < steps; ++it) {
    const long long n = n0 + it;
    const int sn = (int)(n % DL);
    // ---- update -----------------------------------------------------------
    unsigned mask = 0;
    if (tid < qw) {
      const U64x4 v = philox4x64_10((uint64_t)n, (uint64_t)qlocal, 0, kTagDrive, seed, 0);
      const int fslot = (int)(n & kRingMask);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const unsigned pop = (pops >> (8 * k)) & 0xFFu;
        const int jl = 4 * tid + k;
        long long x_int = acc[(size_t)sn * a.B + jl];
        acc[(size_t)sn * a.B + jl] = 0;
        unsigned* fb = &fbits[fslot * a.BW + (jl >> 5)];
        if (*fb & (1u << (jl & 31))) {
          atomicAnd(fb, ~(1u << (jl & 31)));
          x_int += (long long)__hip_atomic_exchange(
              reinterpret_cast<unsigned long long*>(p.ring + (size_t)fslot * p.ring_stride + j0 + jl), 0ull,
              __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (pop == 0xFFu) continue;
        x_int += (long long)poisson_inv(s_table + pop * kTableLen, hi32(pick(v, k))) * p.jext_q;
        const double x = (double)x_int * 0x1p-16;
        const bool free_ = (r[k] == 0);
        if (free_) {
          double yn = p.P22 * y[k] + p.P21 * I[k];
          if (p.i_e != 0.0) yn = yn + p.P20 * p.i_e;
          y[k] = yn;
        } else {
          r[k] = r[k] - 1;
        }
        I[k] = p.P11 * I[k] + x;
        if (free_ && y[k] >= p.theta) {
          y[k] = p.y_reset;
          r[k] = p.ref_steps;
          mask |= 1u << k;
          atomicAdd(&s_popcnt[pop], 1ull);
        }
      }
    }
    // ---- compaction (ascending ids) and publication --------------------------
    int nloc;
    const int c = __popc(mask);
    const int pre = block_exscan(c, s_tmp, &nloc);
    if (mask) {
      int pos = pre;
      for (int k = 0; k < 4; ++k)
        if (mask & (1u << k)) s_local[pos++] = (int)(j0 + 4 * tid + k);
    }
    __syncthreads();
    const int par = (int)(n & 1);
    int* mypub = a.pub + ((size_t)g * 2 + par) * a.B;
    for (int k = tid; k < nloc; k += nthr) {
      __hip_atomic_store(&mypub[k], s_local[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (rcnt + nloc <= p.raster_cap) p.raster[(size_t)g * p.raster_cap + rcnt + k] = make_int2((int)n, s_local[k]);
    }
    if (rcnt + nloc <= p.raster_cap) rcnt += nloc;
    else if (tid == 0) atomicOr(p.overflow, 1u);
    __builtin_amdgcn_s_waitcnt(0);  // ids complete before the flag
    __syncthreads();
    const unsigned long long tag = (unsigned long long)(n + 1);
    if (tid == 0)
      __hip_atomic_store(&a.flags[(size_t)g * kFlagStride], (tag << 32) | (unsigned)nloc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // ---- wait for every workgroup's step-n flag; per-workgroup counts -------
    int cnt_h = 0;
    if (tid < a.G) {
      long long spins = 0;
      unsigned long long f;
      while (true) {
        f = ld_dev(&a.flags[(size_t)tid * kFlagStride]);
        if ((f >> 32) >= tag) break;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > a.spin_limit) { atomicOr(p.overflow, 2u); s_abort = 1; break; }
      }
      cnt_h = (int)(f & 0xFFFFFFFFu);
    }
    int S;
    const int pre_h = block_exscan(cnt_h, s_tmp, &S);   // also a barrier
    if (s_abort) break;
    if (tid < a.G) s_pre[tid] = pre_h;
    if (tid == 0) s_pre[a.G] = S;
    __syncthreads();
    // ---- deliver the step's spikes into my block, kListCap at a time --------
    for (int base = 0; base < S; base += kListCap) {
      const int cnt = min(kListCap, S - base);
      for (int k = tid; k < cnt; k += nthr) {
        const int gk = base + k;
        int lo = 0, hi = a.G;                 // owner workgroup h: s_pre[h] <= gk < s_pre[h+1]
        while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (s_pre[mid] <= gk) lo = mid; else hi = mid; }
        const int i = ld_dev(&a.pub[((size_t)lo * 2 + par) * a.B + (gk - s_pre[lo])]);
        s_list[k] = i;
        const long long* bi = a.blk + (size_t)i * (a.G + 1) + g;
        const long long b0 = bi[0], b1 = bi[1];
        s_lo[k] = b0;
        s_len[k] = (int)(b1 - b0);
      }
      __syncthreads();
      int E;
      const int mylen = (tid < cnt) ? s_len[tid] : 0;
      int ex = block_exscan(mylen, s_tmp, &E);
      // s_len <- exclusive prefix (entries of spikes beyond blockDim handled below)
      if (cnt > nthr) {
        // serial fallback for long lists: thread 0 scans
        __syncthreads();
        if (tid == 0) { int acc_ = 0; for (int k = 0; k < cnt; ++k) { const int l = s_len[k]; s_len[k] = acc_; acc_ += l; } s_tmp[0] = acc_; }
        __syncthreads();
        E = s_tmp[0];
      } else {
        if (tid < cnt) s_len[tid] = ex;
        __syncthreads();
      }
      if (tid == 0) s_events += (unsigned long long)E;
      for (int f = tid; f < E; f += nthr) {
        int lo = 0, hi = cnt;                 // spike k: s_len[k] <= f < s_len[k+1]
        while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (s_len[mid] <= f) lo = mid; else hi = mid; }
        const long long e = s_lo[lo] + (f - s_len[lo]);
        const int t = p.tgt[e];
        const int w = p.wq[e];
        const int d = p.dly[e];
        const int jl = (int)(t - j0);
        if (d < DL) {
          int s = sn + d;
          if (s >= DL) s -= DL;
          atomicAdd(reinterpret_cast<unsigned long long*>(&acc[(size_t)s * a.B + jl]), (unsigned long long)(long long)w);
        } else {
          const int fs = (int)((n + d) & kRingMask);
          atomicAdd(reinterpret_cast<unsigned long long*>(p.ring + (size_t)fs * p.ring_stride + t), (unsigned long long)(long long)w);
          atomicOr(&fbits[fs * a.BW + (jl >> 5)], 1u << (jl & 31));
        }
      }
      __syncthreads();
    }
  }
  // ---- epilogue: state, counters, LDS window back into the global ring ------
  const long long n_end = n0 + steps;
  if (tid < qw) {
    for (int k = 0; k < 4; ++k) { p.y[4 * q + k] = y[k]; p.I[4 * q + k] = I[k]; p.r[4 * q + k] = r[k]; }
  }
  if (tid < p.n_pops) p.wg_spikes[(size_t)g * p.n_pops + tid] += s_popcnt[tid];
  if (tid == 0) {
    p.raster_cnt[g] = rcnt;
    p.wg_events[g] += s_events;
  }
  for (int k = tid; k < DL * Bg; k += nthr) {
    const int m = k / Bg, jl = k - m * Bg;
    const long long step = n_end + m;
    const long long v = acc[(size_t)(step % DL) * a.B + jl];
    if (v != 0)
      atomicAdd(reinterpret_cast<unsigned long long*>(p.ring + (size_t)(step & kRingMask) * p.ring_stride + j0 + jl),
                (unsigned long long)v);
  }
}

__global__ void k_zero_flags(unsigned long long* flags, int n) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) flags[k] = 0;
}

// blk[i][g] = first synapse of row i whose target is >= g*B (rows sorted by target).
__global__ void k_build_blk(const int64_t* row_ptr, const int32_t* tgt, long long n_pad, int G, int B, long long* blk) {
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= n_pad * (G + 1)) return;
  const long long i = idx / (G + 1);
  const int g = (int)(idx - i * (G + 1));
  long long lo = row_ptr[i], hi = row_ptr[i + 1];
  const long long key = (long long)g * B;
  while (lo < hi) { const long long mid = (lo + hi) >> 1; if (tgt[mid] < key) lo = mid + 1; else hi = mid; }
  blk[idx] = lo;
}

size_t persist_lds_bytes(int G, int B, int DL) {
  const int BW = (B + 31) / 32;
  size_t b = (size_t)DL * B * 8 + (size_t)128 * BW * 4 + (size_t)(G + 1) * 4 + (size_t)kListCap * 4 * 2;
  b = (b + 15) & ~(size_t)15;
  b += (size_t)kListCap * 8 + 16;
  return b;
}

hipError_t persist_static_lds(size_t* bytes) {
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, (const void*)k_persist);
  *bytes = (e == hipSuccess) ? attr.sharedSizeBytes : 0;
  return e;
}

hipError_t persist_occupancy(int block, size_t lds, int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_persist, block, lds);
}

hipError_t launch_persist(const DevNet& p, const PersistArgs& a, int steps, int block, hipStream_t s) {
  const size_t lds = persist_lds_bytes(a.G, a.B, a.DL);
  hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(256), 0, s, a.flags, a.G * kFlagStride);
  hipLaunchKernelGGL(k_persist, dim3(a.G), dim3(block), lds, s, p, a, steps);
  return hipGetLastError();
}

hipError_t launch_build_blk(const int64_t* row_ptr, const int32_t* tgt, long long n_pad, int G, int B, long long* blk,
                            hipStream_t s) {
  const long long total = n_pad * (G + 1);
  hipLaunchKernelGGL(k_build_blk, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, row_ptr, tgt, n_pad, G, B, blk);
  return hipGetLastError();
}

hipError_t persist_set_lds_limit(size_t lds) {
  return hipFuncSetAttribute((const void*)k_persist, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

}  // namespace mc
