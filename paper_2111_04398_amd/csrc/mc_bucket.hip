// mc_bucket.hip -- persistent multi-step kernel for many independent
// instances (and any network too large for the LDS window of k_persist):
// target-owner delivery into per-workgroup delay buckets.
//
// Every workgroup owns a block of at most B target neurons of one instance
// (every nthr-th target per thread; the state in LDS) and exchanges spike
// records only with
// the workgroups of its own instance: instances never interact, so a batch
// runs as independent groups inside one launch and a slow instance delays
// only itself.
//
// Why buckets: at the batch's size (7.5e5 neurons) the LDS of a compute unit
// holds only a few steps of pending input for its ~3000 targets, so most
// events would be device-scope int64 atomics into the ring, and those are
// performed at the memory side at ~2e10/s for the whole chip (~50 us per
// step for the batch's ~1.1e6 events).  Instead, the events of a step are
// appended to buckets of the owner workgroup, one bucket per arrival step
// (step mod 128): an LDS counter gives the position, the entry (local
// target, weight) is stored to global memory with a plain (workgroup-scope)
// store, so the L2 gathers a bucket's entries into whole lines.  When the arrival step comes,
// the owner reads its bucket back (one coalesced pass) and sums it in LDS
// with LDS atomics.  The events' global traffic becomes a streaming write
// and a streaming read of 8 bytes each.  The sums are integer sums, so the
// order of the entries does not matter.  A bucket that is full sends further
// events to the global ring with device atomics (the owner reads the ring
// slot of that step too); at the end of a launch the buckets still pending
// are summed into the ring, where the next launch (or another scheme)
// finds them.
//
// Step order per iteration n (as k_persist: the spike decision of step m
// needs I from before step m's input, so step n+1's decision and record go
// out before the wait for step n's records):
//   1. the rest of step n's bucket -> LDS sums; input of step n (+ ring, +
//      drive) into I;
//   2. spike decision of step n+1; compaction; record of step n+1;
//   3. one wavefront waits for the records of step n of the instance's
//      workgroups, listing their spike ids, while the others draw the drive
//      of step n+1 and sum the entries step n+1's bucket already holds (all
//      but those of delay 1, which arrive in 4.);
//   4. every event of step n's spikes that lands in this block goes into the
//      bucket of its arrival step.  The events of a spike that land in the
//      block are one segment of its row; the segment bounds are found at
//      offset (i - first id of the instance) * (blocks of the instance + 1)
//      of the bounds table, so a batch of spikes costs one round of loads.
// Spike records: four per workgroup (step mod 4).  Word 0 = tag16 << 48 |
// count << 36 | the block-local indices (12 bits each) of the first three
// spikes; words 1..3 = (step + 1) << 32 | id of spikes 4..6; later ids in a
// side array written before word 0.  The last workgroup to finish a launch
// clears every record, so a tag needs to carry only the step.
#pragma clang fp contract(off)

#include <algorithm>

#include "mc_device.h"

namespace mc {

namespace {

constexpr int kBW0Ids = 3;              // ids in word 0 (12-bit block-local indices)
constexpr int kBInline = kBW0Ids + 3;   // ids carried by a record
constexpr int kBListCap = 1024;         // spikes of one step listed in LDS (more: chunked, from the records)
constexpr int kBBigCap = 64;            // producers with more than kBInline spikes listed per step
constexpr int kBPollPerLane = kBucketMaxProducers / 64;
constexpr int kBUnroll = 4;             // entries in flight per lane

template <class T>
__device__ __forceinline__ T bld(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void bst(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Bucket entries are written and read back by the same workgroup only (the
// barriers between order them), so workgroup scope suffices: plain cached
// accesses, which the L2 merges into whole lines.
__device__ __forceinline__ unsigned long long wld(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wst(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int bpoisson(const uint64_t* T, uint32_t u) {
  int k = 0;
  while ((uint64_t)u >= T[k]) ++k;
  return k;
}

// Block-wide exclusive scan of one int per thread (s_tmp: one int per wave).
__device__ __forceinline__ int bscan(int v, int* s_tmp, int* total) {
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
  *total = tot;
  return woff + x - v;
}

}  // namespace

__host__ __device__ size_t bucket_sum_slots(int B) { return (size_t)B; }

// LDS (dynamic): s_x[B] i64 (input sums of the step being absorbed) | s_y[B]
// f64 | s_I[B] f64 | s_r[B] i32 | s_kd[B] u8 (Poisson count of the step) |
// s_pop[B] u8.  The neuron state lives in LDS, so registers do not bound the
// block size.
// kRec: the adjoint's forward recording; kTime: phase timestamps.  Plain
// simulation runs the instance with neither (fewer registers in use).
// kBPoll: producers polled per lane (1 when no instance has more than 64
// workgroups, else 8).
template <bool kRec, bool kTime, int kBPoll>
__global__ __launch_bounds__(kBucketMaxBlock) void k_bucket(DevNet p, BucketArgs a, int steps) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  __shared__ uint64_t s_table[kMaxPops * kTableLen];
  __shared__ int s_bcnt[kRingSlots];           // entries in each bucket (arrival step mod 128)
  __shared__ unsigned s_dirty[kRingSlots / 32];  // ring slots that received bucket overflow
  __shared__ int s_tmp[2][16];
  __shared__ int s_first[kBInline];             // ids of the step's first spikes (record)
  __shared__ int s_cnt[kBucketMaxProducers];    // spike count of each producer of the instance this step
  __shared__ int s_hpre[kBucketMaxProducers + 1];  // their prefix (listing of a step beyond the LDS list)
  __shared__ int s_npub;                       // spikes of the step being published
  __shared__ int s_ids[kBListCap];
  __shared__ int2 s_big[kBBigCap];
  __shared__ int s_nids, s_nbig, s_abort, s_last;
  __shared__ unsigned long long s_events;
  __shared__ unsigned long long s_popcnt[kMaxPops];
  const int B = a.B;
  const size_t bx = bucket_sum_slots(B);
  long long* s_x = reinterpret_cast<long long*>(s_raw);
  double* s_y = reinterpret_cast<double*>(s_x + bx);
  double* s_I = s_y + B;
  int* s_r = reinterpret_cast<int*>(s_I + B);
  unsigned char* s_kd = reinterpret_cast<unsigned char*>(s_r + B);
  unsigned char* s_pop = s_kd + B;

  const int g = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
  const int b = a.binst[g], lb = a.blb[g];
  const int gi0 = a.ifb[b];                                        // the instance's first workgroup
  const int Gi = ((b + 1 < p.n_inst) ? a.ifb[b + 1] : a.G) - gi0;   // its workgroups
  const long long j0 = a.bt0[g];
  const int Bg = a.bt0[g + 1] - a.bt0[g];
  // the sources of this instance have Gi + 1 block bounds each, from its first id i0 on
  const int i0 = a.bt0[gi0];
  const int64_t boff0 = a.boff[i0] + lb;
  const long long n0 = *p.step_base;
  unsigned long long* bk = a.bk + (size_t)g * kRingSlots * a.cap;

  for (int k = tid; k < p.n_pops * kTableLen; k += nthr) s_table[k] = p.table[k];
  for (int k = tid; k < (int)bx; k += nthr) s_x[k] = 0;
  for (int k = tid; k < kRingSlots; k += nthr) s_bcnt[k] = 0;
  if (tid < kRingSlots / 32) s_dirty[tid] = 0;
  for (int k = tid; k < kBucketMaxProducers; k += nthr) s_cnt[k] = 0;
  if (tid == 0) { s_abort = 0; s_events = 0; s_npub = 0; }
  if (tid < kMaxPops) s_popcnt[tid] = 0;
  for (int jl = tid; jl < Bg; jl += nthr) {
    const long long j = j0 + jl;
    s_y[jl] = p.y[j]; s_I[jl] = p.I[j]; s_r[jl] = p.r[j];
    s_pop[jl] = (unsigned char)((p.qpops[j >> 2] >> (8 * (j & 3))) & 0xFFu);
    s_kd[jl] = 0;
  }
  __syncthreads();

  // thread t owns local targets t, t + nthr, t + 2 nthr, ... (K rounds):
  // the lanes of a wavefront touch consecutive LDS words, with no bank
  // conflicts (consecutive targets per thread put the lanes 64 bytes apart).
  // Ascending ids go round by round, threads in order.
  const int K = (Bg + nthr - 1) / nthr;
  // Poisson counts of quads q0, q0 + dq, ... at step m (one Philox block per quad)
  auto drive_quads = [&](long long m, int q0, int dq) {
    for (int q4 = 4 * q0; q4 < Bg; q4 += 4 * dq) {
      const long long q = (j0 + q4) >> 2;
      const U64x4 v = philox4x64_10((uint64_t)m, (uint64_t)p.qlocal[q], 0, kTagDrive, p.qseed[q], 0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int jl = q4 + k;
        const unsigned pk = s_pop[jl];
        s_kd[jl] = (pk == 0xFFu) ? 0 : (unsigned char)bpoisson(s_table + pk * kTableLen, hi32(pick(v, (unsigned)k)));
      }
    }
  };
  long long rcnt = p.raster_cnt[g];
  long long ck_seg = -1, ck_phase = 1;
  if (kRec && p.ck_y) {
    const long long k = n0 - p.ck_step0;
    ck_seg = (k >= 0) ? k / p.ck_every : -1;
    ck_phase = (k >= 0) ? k % p.ck_every : 1;
  }
  if (steps > 0) drive_quads(n0, tid, nthr);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  auto decide = [&](long long m) -> uint64_t {   // spike decision of step m: bit k = local target tid + k nthr spiked
    if (kRec && p.ck_y) {
      if (ck_phase == 0 && ck_seg >= 0 && ck_seg < p.ck_count) {
        for (int jl = tid; jl < Bg; jl += nthr) {
          const size_t at = (size_t)ck_seg * p.ring_stride + j0 + jl;
          p.ck_y[at] = s_y[jl]; p.ck_I[at] = s_I[jl]; p.ck_r[at] = s_r[jl];
        }
      }
      if (++ck_phase == p.ck_every) { ck_phase = 0; ++ck_seg; }
    }
    uint64_t mask = 0;
    for (int k = 0; k < K; ++k) {
      const int jl = tid + k * nthr;
      if (jl >= Bg) break;
      const unsigned pk = s_pop[jl];
      if (pk == 0xFFu) continue;
      const int r = s_r[jl];
      const bool free_ = (r == 0);
      double y = s_y[jl];
      if (free_) {
        double yn = p.P22 * y + p.P21 * s_I[jl];
        if (p.i_e != 0.0) yn = yn + p.P20 * p.i_e;
        y = yn;
      }
      if (free_ && y >= p.theta) {
        s_y[jl] = p.y_reset;
        s_r[jl] = p.ref_steps;
        mask |= 1ull << k;
        atomicAdd(&s_popcnt[pk], 1ull);
      } else {
        s_y[jl] = y;
        if (!free_) s_r[jl] = r - 1;
      }
    }
    return mask;
  };
  auto publish = [&](long long m, uint64_t mask) {   // compaction, record of step m, raster
    // slots in any order (delivery sums integers; the raster of a step is
    // ordered on the host): a lane-prefix of the spike counts, one LDS atomic
    // per wavefront for its base
    const int c = __popcll(mask);
    int x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    int wbase = 0;
    if (lane == 63 && x > 0) wbase = atomicAdd(&s_npub, x);
    wbase = __shfl(wbase, 63, 64);
    __syncthreads();
    const int nloc = s_npub;
    const unsigned long long tag = (unsigned long long)(m + 1) << 32;
    const unsigned long long tag16 = (unsigned long long)((m + 1) % 65535 + 1) << 48;
    const size_t rec = (size_t)g * kRecSlots + (size_t)(m % kRecSlots);
    unsigned long long* myrec = a.flags + rec * kPersistFlagStride;
    const bool fits = rcnt + nloc <= p.raster_cap;
    int pos = wbase + x - c;
    for (uint64_t mm = mask; mm; mm &= mm - 1, ++pos) {
      const int id = (int)(j0 + tid + __builtin_ctzll(mm) * nthr);
      if (pos < kBInline) s_first[pos] = id;
      else bst(&a.pub[rec * B + pos], id);
      if (fits) p.raster[(size_t)g * p.raster_cap + rcnt + pos] = make_int2((int)m, id);
    }
    if (nloc > kBInline) __builtin_amdgcn_s_waitcnt(0);   // side-array ids complete before word 0
    __syncthreads();
    if (tid >= kBW0Ids && tid < min(nloc, kBInline)) bst(&myrec[1 + tid - kBW0Ids], tag | (unsigned)s_first[tid]);
    if (tid == 0) {
      unsigned long long w = tag16 | (unsigned long long)nloc << 36;
      for (int k = 0; k < min(nloc, kBW0Ids); ++k) w |= (unsigned long long)(s_first[k] - j0) << (12 * k);
      bst(&myrec[0], w);
      s_npub = 0;                              // read by every thread before the barrier above
    }
    if (fits) rcnt += nloc;
    else if (tid == 0) atomicOr(p.overflow, 1u);
  };
  // id k of producer h's record of step n (after its record has been accepted)
  auto rec_id = [&](int h, size_t rslot, int k) -> int {
    const unsigned long long* rec = a.flags + ((size_t)h * kRecSlots + rslot) * kPersistFlagStride;
    if (k < kBW0Ids) return a.bt0[h] + (int)((bld(&rec[0]) >> (12 * k)) & 0xFFFu);
    if (k < kBInline) return (int)(bld(&rec[1 + k - kBW0Ids]) & 0xFFFFFFFFu);
    return bld(&a.pub[((size_t)h * kRecSlots + rslot) * B + k]);
  };
  // one wavefront appends the events of spikes ids[k0..k1) of step ns that
  // land in this block to the buckets of their arrival steps
  auto deliver = [&](const int* ids, int k0, int k1, long long ns, unsigned long long* ev_out) {
    unsigned long long ev = 0;
    for (int base = k0; base < k1; base += 64) {
      long long lo = 0;
      int len = 0;
      if (base + lane < k1) {
        const int i = ids[base + lane];
        const int64_t o = boff0 + (int64_t)(i - i0) * (Gi + 1);
        const int b0 = a.blk2[o], b1 = a.blk2[o + 1];
        lo = p.row_ptr[i] + b0;
        len = b1 - b0;
        ev += (unsigned long long)len;
      }
      int x = len;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int yv = __shfl_up(x, o, 64);
        if (lane >= o) x += yv;
      }
      const int total = __builtin_amdgcn_readlane(x, 63);   // uniform (an SGPR)
      const int excl = x - len;
      const int lo_lo = (int)(unsigned)(lo & 0xFFFFFFFFll), lo_hi = (int)(lo >> 32);
      // Event f of the batch belongs to the last spike j with excl[j] <= f.
      // The spikes are walked in order by a uniform index (no cross-lane
      // search): js is the spike of the first event of the current chunk
      // of 64, and each lane moves past the segment starts inside its chunk.
      int js = 0;
      for (int f0 = 0; f0 < total; f0 += 64 * kBUnroll) {
        int tt[kBUnroll], ww[kBUnroll], dd[kBUnroll];
#pragma unroll
        for (int u = 0; u < kBUnroll; ++u) {
          const int fb = f0 + u * 64, f = fb + lane;
          dd[u] = 0;
          if (fb < total) {
            while (js < 63 && __builtin_amdgcn_readlane(excl, js + 1) <= fb) ++js;
            int ex_j = __builtin_amdgcn_readlane(excl, js);
            unsigned e_lo = (unsigned)__builtin_amdgcn_readlane(lo_lo, js);
            int e_hi = __builtin_amdgcn_readlane(lo_hi, js);
            for (int jj = js + 1; jj < 64; ++jj) {
              const int ex = __builtin_amdgcn_readlane(excl, jj);
              if (ex > fb + 63) break;
              const unsigned l_lo = (unsigned)__builtin_amdgcn_readlane(lo_lo, jj);
              const int l_hi = __builtin_amdgcn_readlane(lo_hi, jj);
              if (f >= ex) { ex_j = ex; e_lo = l_lo; e_hi = l_hi; }
            }
            if (f < total) {
              const long long e = (long long)(((unsigned long long)(unsigned)e_hi << 32) | e_lo) + (f - ex_j);
              tt[u] = p.tgt[e];
              ww[u] = p.wq[e];
              dd[u] = p.dly[e];
            }
          }
        }
#pragma unroll
        for (int u = 0; u < kBUnroll; ++u) {
          if (dd[u] == 0) continue;
          const int slot = (int)((ns + dd[u]) & kRingMask);
          const int at = atomicAdd(&s_bcnt[slot], 1);
          if (at < a.cap) {
            wst(&bk[(size_t)slot * a.cap + at], (unsigned long long)(unsigned)(tt[u] - j0) << 32 | (unsigned)ww[u]);
          } else {   // full bucket: the ring slot, read by the owner at that step
            atomicAdd(reinterpret_cast<unsigned long long*>(p.ring + (size_t)slot * p.ring_stride + tt[u]),
                      (unsigned long long)(long long)ww[u]);
            atomicOr(&s_dirty[slot >> 5], 1u << (slot & 31));
          }
        }
      }
    }
    *ev_out += ev;
  };

  // entries [from, cnt) of bucket `sl` summed into s_x by threads t of nt,
  // kAbsorb entries in flight per thread
  auto absorb_bucket = [&](int sl, int from, int cnt, int t, int nt) {
    constexpr int kAbsorb = 8;
    const unsigned long long* bq = bk + (size_t)sl * a.cap;
    for (int e0 = from + t; e0 < cnt; e0 += kAbsorb * nt) {
      unsigned long long v[kAbsorb];
#pragma unroll
      for (int u = 0; u < kAbsorb; ++u) v[u] = (e0 + u * nt < cnt) ? wld(&bq[e0 + u * nt]) : 0ull;
#pragma unroll
      for (int u = 0; u < kAbsorb; ++u)
        if (e0 + u * nt < cnt)
          atomicAdd(reinterpret_cast<unsigned long long*>(&s_x[v[u] >> 32]),
                    (unsigned long long)(long long)(int)(v[u] & 0xFFFFFFFFu));
    }
  };

  uint64_t mask = 0;
  if (steps > 0) {
    mask = decide(n0);
    publish(n0, mask);
  }
  long long ph[7] = {0, 0, 0, 0, 0, 0, 0};   // phase ticks (thread 0; [6]: the first polling thread)
  // entries of the bucket of the coming step already summed into s_x while
  // the previous step's records were awaited (the same count in every thread)
  int absorbed = 0;
  for (int it = 0; it < steps; ++it) {
    const long long n = n0 + it;
    const int slot = (int)(n & kRingMask);
    const size_t rslot = (size_t)(n % kRecSlots);
    const bool timing = kTime && tid == 0;
    long long tp0 = timing ? wall_clock64() : 0;
    // ---- 1. input of step n: its bucket summed in LDS, then into I --------
    absorb_bucket(slot, absorbed, min(s_bcnt[slot], a.cap), tid, nthr);
    const bool read_ring = (it < a.horizon) || ((s_dirty[slot >> 5] >> (slot & 31)) & 1u);
    __syncthreads();
    if (tid == 0) {
      s_bcnt[slot] = 0;
      s_dirty[slot >> 5] &= ~(1u << (slot & 31));
      s_nids = 0;
      s_nbig = 0;
    }
    for (int jl = tid; jl < Bg; jl += nthr) {
      long long x_int = s_x[jl];
      s_x[jl] = 0;
      if (read_ring) {
        long long* e = p.ring + (size_t)slot * p.ring_stride + j0 + jl;
        const long long v = bld(e);
        if (v != 0) { bst(e, 0ll); x_int += v; }
      }
      const unsigned pk = s_pop[jl];
      if (pk != 0xFFu) x_int += (long long)s_kd[jl] * p.jext_q;
      if (kRec && p.xrec && n - p.xrec_step0 >= 0 && n - p.xrec_step0 < p.xrec_steps)
        p.xrec[(size_t)(n - p.xrec_step0) * p.ring_stride + j0 + jl] = x_int;
      if (pk != 0xFFu) s_I[jl] = p.P11 * s_I[jl] + (double)x_int * 0x1p-16;
    }
    // ---- 2. spike decision and record of step n+1 ---------------------------
    mask = 0;
    if (it + 1 < steps) {
      mask = decide(n + 1);
      if (timing) { const long long t = wall_clock64(); ph[0] += t - tp0; tp0 = t; }
      publish(n + 1, mask);
    } else {
      if (timing) { const long long t = wall_clock64(); ph[0] += t - tp0; tp0 = t; }
      __syncthreads();
    }
    if (timing) { const long long t = wall_clock64(); ph[1] += t - tp0; tp0 = t; }
    // ---- 3. while one wavefront waits for the instance's records of step n:
    //      the drive of step n+1 and the entries step n+1's bucket already
    //      holds (it gains more only in the delivery below), by the others --
    const int nwork = (nw > 1) ? nthr - 64 : 0;   // threads that do not poll
    const int sl1 = (int)((n + 1) & kRingMask);
    absorbed = (it + 1 < steps && nwork > 0) ? min(s_bcnt[sl1], a.cap) : 0;
    if (tid < nwork && it + 1 < steps) {
      drive_quads(n + 1, tid, nwork);
      absorb_bucket(sl1, 0, absorbed, tid, nwork);
    }
    if (timing) ph[5] += wall_clock64() - tp0;
    const unsigned long long tag = (unsigned long long)(n + 1) << 32;
    const unsigned long long tag16 = (unsigned long long)((n + 1) % 65535 + 1) << 48;
    if (wave == nw - 1) {
      const long long tp_poll = kTime ? wall_clock64() : 0;
      long long t_poll = 0;          // the wall clock is read every 256 rounds only
      unsigned spins = 0;
      unsigned todo = 0;
#pragma unroll
      for (int rr = 0; rr < kBPoll; ++rr)
        if (lane + 64 * rr < Gi) todo |= 1u << rr;
      while (todo) {
        unsigned long long w0[kBPoll];
#pragma unroll
        for (int rr = 0; rr < kBPoll; ++rr)
          w0[rr] = ((todo >> rr) & 1u)
                       ? bld(&a.flags[((size_t)(gi0 + lane + 64 * rr) * kRecSlots + rslot) * kPersistFlagStride])
                       : 0ull;
#pragma unroll
        for (int rr = 0; rr < kBPoll; ++rr) {
          if (!((todo >> rr) & 1u) || (w0[rr] & 0xFFFF000000000000ull) != tag16) continue;
          const int hl = lane + 64 * rr, h = gi0 + hl;
          const int c = (int)((w0[rr] >> 36) & 0xFFFu);
          unsigned long long wk[kBInline - kBW0Ids];
          bool ok = true;
          if (c > kBW0Ids) {
            const unsigned long long* rec = a.flags + ((size_t)h * kRecSlots + rslot) * kPersistFlagStride;
#pragma unroll
            for (int k = 0; k < kBInline - kBW0Ids; ++k) wk[k] = bld(&rec[1 + k]);
#pragma unroll
            for (int k = 0; k < kBInline - kBW0Ids; ++k)
              if (kBW0Ids + k < c) ok &= ((wk[k] & 0xFFFFFFFF00000000ull) == tag);
          }
          if (!ok) continue;
          s_cnt[hl] = c;
          if (c > 0) {
            const int o = atomicAdd(&s_nids, c);
            const int hb = a.bt0[h];
            for (int k = 0; k < min(c, kBInline); ++k) {
              if (o + k >= kBListCap) break;
              s_ids[o + k] = (k < kBW0Ids) ? hb + (int)((w0[rr] >> (12 * k)) & 0xFFFu)
                                           : (int)(wk[k - kBW0Ids] & 0xFFFFFFFFu);
            }
            if (c > kBInline) {
              const int bg = atomicAdd(&s_nbig, 1);
              if (bg < kBBigCap) s_big[bg] = make_int2(h, o);
            }
          }
          todo &= ~(1u << rr);
        }
        if (!todo) break;
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255u) == 0u && (t_poll == 0 ? ((t_poll = wall_clock64()), false) : wall_clock64() - t_poll > a.wait_ticks)) {
          atomicOr(p.overflow, 2u);
          s_abort = 1;
#pragma unroll
          for (int rr = 0; rr < kBPoll; ++rr)
            if ((todo >> rr) & 1u) s_cnt[lane + 64 * rr] = 0;
          break;
        }
      }
      if (kTime && tid == nthr - 64) ph[6] += wall_clock64() - tp_poll;
      if (nwork == 0 && it + 1 < steps) drive_quads(n + 1, tid, nthr);   // a one-wavefront block
    }
    __syncthreads();
    if (timing) { const long long t = wall_clock64(); ph[2] += t - tp0; tp0 = t; }
    if (s_abort) break;
    // ---- 4. events of step n's spikes into the buckets ----------------------
    const int S = s_nids;
    unsigned long long ev = 0;
    if (S <= kBListCap && s_nbig <= kBBigCap) {
      const int nbig = s_nbig;
      if (nbig > 0) {
        for (int e = 0; e < nbig; ++e) {
          const int h = s_big[e].x, o = s_big[e].y, c = s_cnt[h - gi0];
          for (int k = kBInline + tid; k < c; k += nthr) s_ids[o + k] = bld(&a.pub[((size_t)h * kRecSlots + rslot) * B + k]);
        }
        __syncthreads();
      }
      if (timing) { const long long t = wall_clock64(); ph[3] += t - tp0; tp0 = t; }
      const int k0 = (int)((long long)S * wave / nw), k1 = (int)((long long)S * (wave + 1) / nw);
      deliver(s_ids, k0, k1, n, &ev);
    } else {
      // more spikes than the list holds: in producer order, chunk by chunk,
      // the ids read again from the records (thread t sums producers 2t, 2t+1)
      const int c0 = (2 * tid < Gi) ? s_cnt[2 * tid] : 0;
      const int c1 = (2 * tid + 1 < Gi) ? s_cnt[2 * tid + 1] : 0;
      int Sall;
      const int pre_h = bscan(c0 + c1, s_tmp[1], &Sall);
      __syncthreads();
      int* s_pre = s_hpre;
      if (2 * tid < Gi) s_pre[2 * tid] = pre_h;
      if (2 * tid + 1 < Gi) s_pre[2 * tid + 1] = pre_h + c0;
      if (tid == 0) s_pre[Gi] = Sall;
      __syncthreads();
      for (int base = 0; base < Sall; base += kBListCap) {
        const int cnt = min(kBListCap, Sall - base);
        for (int k = tid; k < cnt; k += nthr) {
          const int gk = base + k;
          int lo = 0, hi = Gi;
          while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (s_pre[mid] <= gk) lo = mid; else hi = mid; }
          s_ids[k] = rec_id(gi0 + lo, rslot, gk - s_pre[lo]);
        }
        __syncthreads();
        const int k0 = (int)((long long)cnt * wave / nw), k1 = (int)((long long)cnt * (wave + 1) / nw);
        deliver(s_ids, k0, k1, n, &ev);
        __syncthreads();
      }
    }
    if (ev) atomicAdd(&s_events, ev);
    __syncthreads();
    if (timing) ph[4] += wall_clock64() - tp0;
  }
  if (kTime && tid == 0) {
    for (int k = 0; k < 6; ++k) a.phase[(size_t)g * 8 + k] += (unsigned long long)ph[k];
    a.phase[(size_t)g * 8 + 7] += (unsigned long long)steps;
  }
  if (kTime && tid == nthr - 64) a.phase[(size_t)g * 8 + 6] += (unsigned long long)ph[6];
  // ---- epilogue: state, counters; pending buckets summed into the ring -----
  for (int jl = tid; jl < Bg; jl += nthr) { const long long j = j0 + jl; p.y[j] = s_y[jl]; p.I[j] = s_I[jl]; p.r[j] = s_r[jl]; }
  if (tid < p.n_pops) p.wg_spikes[(size_t)g * p.n_pops + tid] += s_popcnt[tid];
  if (tid == 0) {
    p.raster_cnt[g] = rcnt;
    p.wg_events[g] += s_events;
  }
  // (after an abandoned wait s_x may hold part of the next bucket: start from zero)
  for (int jl = tid; jl < Bg; jl += nthr) s_x[jl] = 0;
  __syncthreads();
  for (int sl = 0; sl < kRingSlots; ++sl) {
    if (s_bcnt[sl] == 0) continue;               // uniform: every thread reads the same count
    absorb_bucket(sl, 0, min(s_bcnt[sl], a.cap), tid, nthr);
    __syncthreads();
    for (int jl = tid; jl < Bg; jl += nthr) {
      const long long v = s_x[jl];
      if (v == 0) continue;
      s_x[jl] = 0;
      long long* e = p.ring + (size_t)sl * p.ring_stride + j0 + jl;
      bst(e, bld(e) + v);                        // only this workgroup touches its targets' entries
    }
    __syncthreads();
  }
  // the last workgroup to finish clears the records and advances the step
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    unsigned long long* done = a.flags + persist_record_words(a.G);
    s_last = (__hip_atomic_fetch_add(done, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (unsigned long long)(a.G - 1));
  }
  __syncthreads();
  if (s_last) {
    const int words = (int)persist_record_words(a.G);
    for (int k = tid; k < words; k += nthr) bst(&a.flags[k], 0ull);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      bst(p.step_base, n0 + (long long)steps);
      __hip_atomic_store(a.flags + persist_record_words(a.G), 0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Dynamic LDS of a block of B targets: the input sums (room also for the
// fallback listing's producer prefix), then y, I, r, the step's Poisson
// counts and the populations.
size_t bucket_lds_bytes(int B) {
  return bucket_sum_slots(B) * sizeof(long long) + (size_t)B * (8 + 8 + 4 + 1 + 1);
}

// The instances of k_bucket (recording, timing, poll width); shapes are
// checked against all of them.
const void* const kBucketFns[8] = {
    (const void*)k_bucket<false, false, 1>, (const void*)k_bucket<true, false, 1>,
    (const void*)k_bucket<false, true, 1>,  (const void*)k_bucket<true, true, 1>,
    (const void*)k_bucket<false, false, kBPollPerLane>, (const void*)k_bucket<true, false, kBPollPerLane>,
    (const void*)k_bucket<false, true, kBPollPerLane>,  (const void*)k_bucket<true, true, kBPollPerLane>};

template <bool kRec, bool kTime>
static void launch_bucket_as(const DevNet& p, const BucketArgs& a, int steps, int block, hipStream_t s) {
  auto* const kf = (a.inst_wg_max <= 64) ? k_bucket<kRec, kTime, 1> : k_bucket<kRec, kTime, kBPollPerLane>;
  hipLaunchKernelGGL(kf, dim3(a.G), dim3(block), bucket_lds_bytes(a.B), s, p, a, steps);
}

hipError_t launch_bucket(const DevNet& p, const BucketArgs& a, int steps, int block, hipStream_t s) {
  // a thread owns at most 64 targets (its spike mask), so B <= 64 threads
  if (a.B < 4 || a.B > 64 * block) return hipErrorInvalidValue;
  const bool rec = p.xrec != nullptr || p.ck_y != nullptr, tim = a.phase != nullptr;
  if (rec && tim) launch_bucket_as<true, true>(p, a, steps, block, s);
  else if (rec) launch_bucket_as<true, false>(p, a, steps, block, s);
  else if (tim) launch_bucket_as<false, true>(p, a, steps, block, s);
  else launch_bucket_as<false, false>(p, a, steps, block, s);
  return hipGetLastError();
}

hipError_t bucket_occupancy(int B, int block, int inst_wg_max, int* blocks_per_cu) {
  *blocks_per_cu = 1 << 30;
  const int first = (inst_wg_max <= 64) ? 0 : 4;   // the poll width launch_bucket picks
  for (int k = first; k < first + 4; ++k) {
    const void* f = kBucketFns[k];
    int occ = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, block, bucket_lds_bytes(B));
    if (e != hipSuccess) return e;
    *blocks_per_cu = std::min(*blocks_per_cu, occ);
  }
  return hipSuccess;
}

hipError_t bucket_set_lds_limit(size_t lds) {
  for (const void* f : kBucketFns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mc
