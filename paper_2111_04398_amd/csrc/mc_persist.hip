// mc_persist.hip -- persistent multi-step kernel with the near-future input
// held in LDS (target-owner delivery).
//
// Why: on gfx950 a device-scope int64 atomic is performed at the memory side
// at about 20e9 per second for the whole chip, whatever the footprint of the
// table, so a step of the full microcircuit (~2.5e5 synaptic events) cannot
// drop below ~12 us if every event is a global atomic.  Here every workgroup
// owns a contiguous block of B target neurons (one per thread) and keeps
// their pending input for the next D_L steps in LDS (int64, LDS atomics); it
// delivers, for every spike, only the part of the source row that targets its
// own block (rows are sorted by target, so that part is contiguous and an
// index blk[i][g] gives its bounds).  Events with a delay >= D_L (the tail of
// the delay distribution) go to the global ring with device atomics, into
// entries only the owner reads.  The only cross-workgroup traffic per step is
// the spike list.
//
// Critical path.  Only the events of step n with delay 1 must be in place
// before the input of step n+1 enters I, and those with delay 2 before step
// n+2's.  (The spike decision of a step needs I from before the step, so it
// runs one step earlier: see the loop.)
// Both come from a "near" table (the delay-1/2 synapses per source and
// workgroup, as a CSR), delivered as the spike list of step n fills (the
// first ids while the poll goes on, the rest once the list is complete).  The other events are pipelined over the two following steps,
// while the workgroup waits for the next spike lists: in step n+1 the block
// bounds blk[i][g] of step n's spikes are loaded, in step n+2 their entries
// (delay >= 3, landing at step n+3 or later) are added.  The poller lists the
// ids of each record as it arrives, so the list is complete when the wait
// ends.
//
// Wavefront roles within a step.  Only the wavefronts that hold owned
// targets update, spike and publish; they meet for the compaction on an LDS
// arrival count instead of a block barrier.  The poller (the last wavefront)
// and the wavefronts without targets therefore start at the top of the
// step: the poller polls, the others take items of the pipelined delivery
// (entries of 16 spikes, block bounds of 64) from an LDS counter, and the
// updating wavefronts join the claiming once their record is out.  In a
// quiet step the memory round trips of the pipelined delivery thus overlap
// the update and the publication instead of following them.  The last
// wavefront without targets then adds the near events of the first ids the
// poller lists (at most kEarlyNear) while the poll goes on; a step that
// turns out to need the whole-step fallback takes them out again (the same
// events with the opposite sign: integer sums cancel exactly) first.
//
// Spike exchange: workgroup g publishes a record per step (four per
// workgroup, by step mod 4, so a record is never rewritten while a consumer
// one step behind may still read it).  Compaction is one ballot per
// wavefront (kept in LDS by step parity): a spike's position is the number
// of spikes of lower threads; the first 39 spikes go into the record's
// words (composed from the ballots by lanes 0..7 of wavefront 0), the rest
// each spiking thread stores into the side array.  Word 0 = tag16 << 48 |
// count << 36 | the block-local indices (9 bits each) of the first four
// spikes, with tag16 = (step + 1) mod 65535 + 1 (never 0, distinct for
// consecutive steps); word L = 1..7 = tag16 << 48 | the indices of spikes
// 5L..5L+4.  About four in five workgroups publish no spike in a step and
// nearly all others at most four, so one load of word 0 usually completes a
// record, and the records of a burst carry up to 39 ids without a side array.  Every word carries
// a tag, so a consumer accepts a record when all the words it needs show the
// current step, whatever order the stores became visible in; a tag is the
// step alone, which suffices because the last workgroup to finish a launch
// clears every record, so that no record outlives the launch that wrote it
// (also across rewinds of the state to earlier steps).  Spikes beyond
// the 39th are written to a side array before word 0 (with a wait for
// their completion), so they are visible once word 0 is.  All of these are
// device-scope atomic accesses (coherent at the memory side), so the step
// needs no L2 writeback or invalidate.  Every wait is bounded in time (wall
// clock); on timeout the kernel sets error bit 2 and every workgroup leaves
// the loop.
#pragma clang fp contract(off)

#include <algorithm>
#include "mc_device.h"

namespace mc {

namespace {

constexpr int kListCap = 1024;       // spikes of one step kept in LDS (more: delivered at once)
constexpr int kW0Ids = 4;            // spike ids in word 0 of a record (9-bit block-local indices)
constexpr int kWIds = 5;             // in each of words 1..7
constexpr int kInline = kW0Ids + (kPersistFlagStride - 1) * kWIds;   // 39 carried by a record (more: side array)
constexpr int kBigCap = 64;          // producers with more than kInline spikes listed per step
constexpr int kEarlyNear = 64;       // ids near-delivered during the poll at most (all waves share the rest)
constexpr int kItemSpikes = 16;      // spikes per claimed item of pipelined entries (~ one 256-entry chunk)
constexpr int kUnroll = 4;           // entries in flight per lane
constexpr unsigned kNearD2 = 0x80000000u;   // near-table flag: delay 2 (else 1)

// Workgroups are dispatched to the XCDs round robin (workgroup g runs on XCD
// g mod 8), and each XCD has its own L2.  Per-source tables indexed by
// workgroup are laid out by XCD, so that the entries the workgroups of one
// XCD read for a source share cache lines: position of workgroup g, and its
// inverse.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_pos(int g, int G) {
  const int x = g % kXcds;
  int pos = g / kXcds;
  for (int y = 0; y < x; ++y) pos += (G - y + kXcds - 1) / kXcds;
  return pos;
}
__device__ __forceinline__ int xcd_wg(int pos, int G) {
  for (int x = 0;; ++x) {
    const int c = (G - x + kXcds - 1) / kXcds;
    if (pos < c) return pos * kXcds + x;
    pos -= c;
  }
}

__device__ __forceinline__ int poisson_inv(const uint64_t* T, uint32_t u) {
  int k = 0;
  while ((uint64_t)u >= T[k]) ++k;
  return k;
}

template <class T>
__device__ __forceinline__ T ld_dev(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void st_dev(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-wide exclusive scan of v (one value per thread); returns the
// thread's exclusive prefix, *total the block sum.  s_tmp: one int per wave,
// alternated by the caller between consecutive scans (one barrier each).
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
  *total = tot;
  return woff + x - v;
}

// Poisson counts of the four neurons of a quad at step n, packed in bytes.
__device__ __forceinline__ uint32_t drive_counts(long long n, uint32_t qlocal, uint64_t seed, uint32_t pops,
                                                 const uint64_t* s_table) {
  const U64x4 v = philox4x64_10((uint64_t)n, (uint64_t)qlocal, 0, kTagDrive, seed, 0);
  uint32_t out = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned pop = (pops >> (8 * k)) & 0xFFu;
    if (pop == 0xFFu) continue;
    out |= (uint32_t)poisson_inv(s_table + pop * kTableLen, hi32(pick(v, k))) << (8 * k);
  }
  return out;
}

// Per-workgroup view of the LDS ring and where events of a step go.
struct Block {
  long long* acc;        // [DL][B]
  unsigned* fbits;       // [128][BW]
  int B, BW, DL;
  long long j0;          // first owned (padded) target
};

// Adds one event (target t, weight w, delay d) of a spike at step ns, whose
// LDS slot is sns = ns mod DL, to the owned block.
__device__ __forceinline__ void add_event(const DevNet& p, const Block& b, int t, int w, int d, long long ns, int sns) {
  const int jl = (int)(t - b.j0);
  if (d < b.DL) {
    int s = sns + d;
    if (s >= b.DL) s -= b.DL;
    atomicAdd(reinterpret_cast<unsigned long long*>(&b.acc[(size_t)s * b.B + jl]), (unsigned long long)(long long)w);
  } else {
    const int fs = (int)((ns + d) & kRingMask);
    atomicAdd(reinterpret_cast<unsigned long long*>(p.ring + (size_t)fs * p.ring_stride + t), (unsigned long long)(long long)w);
    atomicOr(&b.fbits[fs * b.BW + (jl >> 5)], 1u << (jl & 31));
  }
}

// One wavefront walks the entries of spikes k0..k1 of step ns, given each
// spike's block bounds (lo, len) through `bounds(k, &lo, &len)`, and adds the
// events with delay >= dmin.  Lanes hold the bounds of 64 spikes, scan their
// lengths, and walk the concatenated entries kUnroll at a time.
template <class Bounds>
__device__ __forceinline__ void wave_entries(const DevNet& p, const Block& b, int k0, int k1, long long ns, int sns,
                                             int dmin, Bounds bounds) {
  const int lane = threadIdx.x & 63;
  for (int base = k0; base < k1; base += 64) {
    long long lo = 0;
    int len = 0;
    if (base + lane < k1) bounds(base + lane, &lo, &len);
    int x = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    const int total = __shfl(x, 63, 64);
    const int excl = x - len;
    for (int f0 = 0; f0 < total; f0 += 64 * kUnroll) {
      int tt[kUnroll], ww[kUnroll], dd[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int f = f0 + u * 64 + lane;
        dd[u] = 0;
        int lo_l = 0, hi_l = 64;              // lane j holding entry f: excl_j <= f < excl_{j+1}
#pragma unroll
        for (int s = 0; s < 6; ++s) {
          const int mid = (lo_l + hi_l) >> 1;
          const int em = __shfl(excl, mid, 64);
          if (em <= f) lo_l = mid; else hi_l = mid;
        }
        const long long lo_j = __shfl(lo, lo_l, 64);
        const int ex_j = __shfl(excl, lo_l, 64);
        if (f < total) {
          const long long e = lo_j + (f - ex_j);
          tt[u] = p.tgt[e];
          ww[u] = p.wq[e];
          dd[u] = p.dly[e];
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u)
        if (dd[u] >= dmin) add_event(p, b, tt[u], ww[u], dd[u], ns, sns);
    }
  }
}

// One wavefront adds the delay-1 and delay-2 events of spikes list[k0..k1)
// that land in this workgroup's block: the near table holds them per
// (source, workgroup) as a CSR over workgroups in XCD order (offsets
// nb[i][p], nb[i][p+1] at the workgroup's position p; entries
// (delay-2 flag | local target) << 32 | weight).  Lanes load the offsets of 64
// spikes, scan the counts and walk the concatenated entries.
__device__ __forceinline__ void wave_near(const PersistArgs& a, const Block& b, const int* list, int k0, int k1, int gpos,
                                          int slot1, int slot2, int sign = 1) {
  const int lane = threadIdx.x & 63;
  for (int base = k0; base < k1; base += 64) {
    unsigned lo = 0;
    int len = 0;
    if (base + lane < k1) {
      const unsigned* o = a.nb + (size_t)list[base + lane] * (a.G + 1) + gpos;
      lo = o[0];
      len = (int)(o[1] - lo);
    }
    int x = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    const int total = __shfl(x, 63, 64);
    const int excl = x - len;
    for (int f0 = 0; f0 < total; f0 += 64 * kUnroll) {
      unsigned long long v[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int f = f0 + u * 64 + lane;
        int lo_l = 0, hi_l = 64;              // lane j holding entry f: excl_j <= f < excl_{j+1}
#pragma unroll
        for (int st = 0; st < 6; ++st) {
          const int mid = (lo_l + hi_l) >> 1;
          if (__shfl(excl, mid, 64) <= f) lo_l = mid; else hi_l = mid;
        }
        const unsigned lo_j = (unsigned)__shfl((int)lo, lo_l, 64);
        const int ex_j = __shfl(excl, lo_l, 64);
        v[u] = (f < total) ? a.ne[lo_j + (unsigned)(f - ex_j)] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        if (f0 + u * 64 + lane >= total) continue;
        const unsigned hi = (unsigned)(v[u] >> 32);
        const int slot = (hi & kNearD2) ? slot2 : slot1;
        atomicAdd(reinterpret_cast<unsigned long long*>(&b.acc[(size_t)slot * b.B + (hi & 0xFFFFu)]),
                  (unsigned long long)((long long)(int)(v[u] & 0xFFFFFFFFu) * sign));
      }
    }
  }
}

}  // namespace

// LDS (dynamic): acc[DL*B] i64 | fbits[128*BW] u32 | s_pre[G+1] | s_ids[2][kListCap]
//                | s_len[2][kListCap] | s_lo[2][kListCap] i64
// kRec: the adjoint's forward recording (input x and state checkpoints);
// kTime: phase timestamps.  Plain simulation runs the instance with neither,
// whose smaller register footprint shortens the step (fewer scalar
// registers spilled to vector lanes).  kPoll: producers polled per lane (4
// when G <= 256: a smaller poll loop, fewer registers; else 8).
template <bool kRec, bool kTime, int kPoll>
__global__ __launch_bounds__(kPersistMaxBlock) void k_persist(DevNet p, PersistArgs a, int steps) {
  extern __shared__ __align__(16) unsigned char s_raw[];
  __shared__ uint64_t s_table[kMaxPops * kTableLen];
  __shared__ int s_tmp[2][16];
  __shared__ uint64_t s_mask[2][kPersistMaxBlock / 64];   // spike ballots per wavefront, by step parity
  __shared__ int s_cnt[kPersistMaxBlock];   // spike count of every producer in the current step
  __shared__ int s_abort, s_last;
  __shared__ int s_nids, s_nbig;                 // ids listed by the poller this step; producers with more
  __shared__ int2 s_big[kBigCap];                // (producer, list offset) of those producers
  __shared__ unsigned long long s_events;
  __shared__ int s_work;                         // next item of the step's pipelined delivery
  __shared__ int s_pubcnt, s_sidecnt;            // arrivals of the updating wavefronts (monotonic)
  __shared__ int s_nready, s_polldone, s_ndone;  // ids listed in complete rounds; poll over; ids near-delivered early
  __shared__ unsigned long long s_popcnt[kMaxPops];
  long long* acc = reinterpret_cast<long long*>(s_raw);
  unsigned* fbits = reinterpret_cast<unsigned*>(acc + (size_t)a.DL * a.B);
  int* s_pre = reinterpret_cast<int*>(fbits + 128 * a.BW);        // [G+1]
  int* s_ids = s_pre + (a.G + 1);                                   // [2][kListCap] spike ids by step parity
  int* s_len = s_ids + 2 * kListCap;                                // [2][kListCap] block sub-row lengths
  long long* s_lo = reinterpret_cast<long long*>(((uintptr_t)(s_len + 2 * kListCap) + 15) & ~(uintptr_t)15);

  const int g = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
  const int gpos = xcd_pos(g, a.G);                                 // column of this workgroup in the near table
  const int wave = tid >> 6, nw = nthr >> 6;
  const long long j0 = a.bstart[g];                                 // first owned target (padded id)
  const int Bg = a.bstart[g + 1] - a.bstart[g];                     // owned targets (multiple of 4, <= B)
  const long long n0 = *p.step_base;
  const int DL = a.DL;
  // the listing threshold (a test hook, read by the phase-timing instance only)
  const int list_cap = (kTime && a.list_cap > 0 && a.list_cap < kListCap) ? a.list_cap : kListCap;
  // Polling: the last wavefront polls every producer workgroup (lane l takes
  // producers l, l+64, ...); the other wavefronts work on the pipelined
  // delivery meanwhile.  A one-wavefront workgroup polls, then works.
  const bool overlap = nw > 1;
  const bool pollw = overlap ? (wave == nw - 1) : true;
  auto par_m = [](long long m) { return (int)(m & 1); };
  const Block blk{acc, fbits, a.B, a.BW, DL, j0};
  auto bounds_of = [&](int par_) {
    return [=](int k, long long* lo, int* len) { *lo = s_lo[par_ * kListCap + k]; *len = s_len[par_ * kListCap + k]; };
  };

  for (int k = tid; k < p.n_pops * kTableLen; k += nthr) s_table[k] = p.table[k];
  for (int k = tid; k < DL * a.B; k += nthr) acc[k] = 0;
  for (int k = tid; k < 128 * a.BW; k += nthr) fbits[k] = 0;
  if (tid == 0) { s_abort = 0; s_events = 0; s_work = 0; s_pubcnt = 0; s_sidecnt = 0; s_nready = 0; s_polldone = 0; s_ndone = 0; }
  if (tid < kMaxPops) s_popcnt[tid] = 0;
  __syncthreads();
  // neuron state into registers: thread t < Bg owns neuron j0+t; the four
  // threads of a quad draw the same Philox block and take their own word
  double y = 0.0, I = 0.0;
  int r = 0;
  unsigned pop = 0xFFu;
  uint32_t qlocal = 0, qpops = 0xFFFFFFFFu;
  int kdrive = 0;
  uint64_t seed = 0;
  const bool upd = tid < Bg;
  // Wavefronts holding owned targets update, spike and publish; they meet
  // for the publication on an LDS arrival count, not a block barrier, so the
  // poller and the wavefronts without targets start the step's waiting work
  // (polling, pipelined delivery) at its top.
  const int nupd_w = (Bg + 63) >> 6;
  const bool updw = wave < nupd_w;
  int pub_epoch = 0, side_epoch = 0;
  auto upd_sync = [&](int* cnt, int& epoch) {
    ++epoch;
    if ((tid & 63) == 0) __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    const int target = epoch * nupd_w;
    long long t_sp = 0;
    unsigned spins = 0;
    while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023u) == 0u &&
          (t_sp == 0 ? ((t_sp = wall_clock64()), false) : wall_clock64() - t_sp > a.wait_ticks)) {
        atomicOr(p.overflow, 2u);
        s_abort = 1;
        break;
      }
    }
  };
  const long long q = (j0 + tid) >> 2;
  const int qk = tid & 3;
  __syncthreads();
  if (upd) {
    qpops = p.qpops[q]; qlocal = p.qlocal[q]; seed = p.qseed[q];
    pop = (qpops >> (8 * qk)) & 0xFFu;
    y = p.y[j0 + tid]; I = p.I[j0 + tid]; r = p.r[j0 + tid];
    if (steps > 0) kdrive = (int)((drive_counts(n0, qlocal, seed, qpops, s_table) >> (8 * qk)) & 0xFFu);
  }
  // first owned target of each producer this lane polls (word 0 carries block-local indices)
  int pbs[kPoll];
#pragma unroll
  for (int r = 0; r < kPoll; ++r) {
    const int h = (tid & 63) + 64 * r;
    pbs[r] = (h < a.G) ? a.bstart[h] : 0;
  }
  long long rcnt = p.raster_cnt[g];
  // checkpoint schedule of an adjoint's forward: segment of step n0 and n0's
  // phase in it (a checkpoint is due at phase 0)
  long long ck_seg = -1, ck_phase = 1;
  if (kRec && p.ck_y) {
    const long long k = n0 - p.ck_step0;
    ck_seg = (k >= 0) ? k / p.ck_every : -1;
    ck_phase = (k >= 0) ? k % p.ck_every : 1;
  }
  long long ph[7] = {0, 0, 0, 0, 0, 0, 0};
  int S1 = 0;                           // spikes of step n-1: ids kept, block bounds due
  int S2 = 0;                           // spikes of step n-2: bounds kept, entries due
  int sn = (int)(n0 % DL);              // LDS slot of the current step
  // every load above has landed: the loop body then waits only for its own
  // memory operations (without this the compiler's wait insertion assumes the
  // initial loads may still be in flight at every iteration and waits for all
  // outstanding operations, stores included, at their first use)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // The update of step m splits in two.  Its spike decision moves y and r
  // with the I of before the step, so it does not need the input read at
  // step m; only I = P11 I + x does.  The spike decision of step m+1 and its
  // record therefore go out before the wait for step m's records, and every
  // workgroup can run up to one step ahead of the slowest.
  auto decide = [&](long long m) -> int {     // spike decision of step m
    if (kRec && p.ck_y) {                   // adjoint forward: checkpoint before the update
      if (upd && ck_phase == 0 && ck_seg >= 0 && ck_seg < p.ck_count) {
        const size_t at = (size_t)ck_seg * p.ring_stride + j0 + tid;
        p.ck_y[at] = y; p.ck_I[at] = I; p.ck_r[at] = r;
      }
      if (++ck_phase == p.ck_every) { ck_phase = 0; ++ck_seg; }
    }
    int spiked = 0;
    if (upd && pop != 0xFFu) {
      const bool free_ = (r == 0);
      if (free_) {
        double yn = p.P22 * y + p.P21 * I;
        if (p.i_e != 0.0) yn = yn + p.P20 * p.i_e;
        y = yn;
      } else {
        r = r - 1;
      }
      if (free_ && y >= p.theta) {
        y = p.y_reset;
        r = p.ref_steps;
        spiked = 1;
        atomicAdd(&s_popcnt[pop], 1ull);
      }
    }
    return spiked;
  };
  auto absorb = [&](long long m, int slot) {  // input of step m into I; its LDS slot cleared
    if (!upd) return;
    const int fslot = (int)(m & kRingMask);
    const int jl = tid;
    long long x_int = acc[(size_t)slot * a.B + jl];
    acc[(size_t)slot * a.B + jl] = 0;
    unsigned* fb = &fbits[fslot * a.BW + (jl >> 5)];
    if (*fb & (1u << (jl & 31))) {
      atomicAnd(fb, ~(1u << (jl & 31)));
      x_int += (long long)__hip_atomic_exchange(
          reinterpret_cast<unsigned long long*>(p.ring + (size_t)fslot * p.ring_stride + j0 + jl), 0ull,
          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (pop != 0xFFu) x_int += (long long)kdrive * p.jext_q;
    if (kRec && p.xrec && m - p.xrec_step0 >= 0 && m - p.xrec_step0 < p.xrec_steps)
      p.xrec[(size_t)(m - p.xrec_step0) * p.ring_stride + j0 + jl] = x_int;
    if (pop != 0xFFu) I = p.P11 * I + (double)x_int * 0x1p-16;
  };
  // t16m = (m + 1) mod 65535 + 1, kept by the caller as a running count
  auto publish = [&](long long m, int spiked, unsigned t16m) {   // compaction (ascending ids), record of step m, raster
    // one ballot per wavefront; a spike's position is the count of spikes of
    // lower threads (thread order = id order)
    const uint64_t bal = __ballot(spiked);
    if ((tid & 63) == 0) s_mask[par_m(m)][wave] = bal;
    upd_sync(&s_pubcnt, pub_epoch);
    const uint64_t* msk = s_mask[par_m(m)];
    uint64_t mr[kPersistMaxBlock / 64];      // the masks, read once into registers
#pragma unroll
    for (int w = 0; w < kPersistMaxBlock / 64; ++w) mr[w] = (w < nupd_w) ? msk[w] : 0ull;
    int nloc = 0, pos = 0;
#pragma unroll
    for (int w = 0; w < kPersistMaxBlock / 64; ++w) {
      const int c = __popcll(mr[w]);
      pos += (w < wave) ? c : 0;
      nloc += c;
    }
    pos += __popcll(bal & ((tid & 63) ? (~0ull >> (64 - (tid & 63))) : 0ull));
    const unsigned long long tag16 = (unsigned long long)t16m << 48;
    const size_t rec = (size_t)g * kRecSlots + (size_t)(m & (kRecSlots - 1));
    unsigned long long* myrec = a.flags + rec * kPersistFlagStride;
    const bool fits = rcnt + nloc <= p.raster_cap;
    if (spiked) {
      const int id = (int)(j0 + tid);
      if (pos >= kInline) st_dev(&a.pub[rec * a.B + pos], id);
      if (fits) p.raster[(size_t)g * p.raster_cap + rcnt + pos] = make_int2((int)m, id);
    }
    if (nloc > kInline) {                   // side-array ids complete before word 0
      __builtin_amdgcn_s_waitcnt(0);
      upd_sync(&s_sidecnt, side_epoch);
    }
    // word L (lanes 0..7 of wavefront 0): word 0 the count and the block-local
    // indices of spikes 1..4, word L >= 1 those of spikes 5L..5L+4; each word
    // carries the step tag
    if (tid < kPersistFlagStride) {
      const int L = tid;
      const int first = (L == 0) ? 0 : kW0Ids + (L - 1) * kWIds, nf = (L == 0) ? kW0Ids : kWIds;
      if (L == 0 || nloc > first) {
        unsigned long long wv = tag16 | ((L == 0) ? (unsigned long long)nloc << 36 : 0ull);
        int seen = 0, f = 0;
#pragma unroll
        for (int w = 0; w < kPersistMaxBlock / 64; ++w) {
          uint64_t mm = mr[w];
          const int cw = __popcll(mm);
          if (seen + cw <= first) { seen += cw; continue; }
          while (mm && f < nf) {
            if (seen >= first) {
              wv |= (unsigned long long)(64 * w + __builtin_ctzll(mm)) << (9 * f);
              ++f;
            }
            ++seen;
            mm &= mm - 1;
          }
        }
        st_dev(&myrec[L], wv);
      }
    }
    if (fits) rcnt += nloc;
    else if (tid == 0) atomicOr(p.overflow, 1u);
  };

  static_assert((kRecSlots & (kRecSlots - 1)) == 0, "record slots by step & (kRecSlots - 1)");
  auto next16 = [](unsigned t) { return t == 65535u ? 1u : t + 1u; };
  unsigned t16n = (unsigned)((n0 + 1) % 65535 + 1);   // tag of step n0's record; advanced every step
  if (steps > 0 && updw) {                    // step n0's spike decision and record
    const int sp = decide(n0);
    publish(n0, sp, t16n);
  }
  // Then take the next DL steps of pending input of my targets into LDS and
  // mark far entries (step n0's decision does not need them, so every
  // workgroup's first record is out while this scan runs).  Only the first
  // `horizon` slots can hold input (the largest delay, or further after an
  // injection or a loaded state).  Inside a launch only the owner workgroup
  // touches its targets' ring entries, so device-scope loads and stores
  // suffice (no read-modify-write).
  // Element (m, jl) is ring slot m ahead of step n0, owned target jl; each
  // thread steps through the elements nthr at a time, carrying (m, jl) along
  // so the slot arithmetic stays in 32 bits (a division per element costs
  // more than its load).
  if (Bg > 0) {
    const int take = min(DL, a.horizon), scan = min(127, a.horizon);
    const int sl0 = (int)(n0 % DL), rs0 = (int)(n0 & kRingMask);   // LDS and ring slot of step n0
    const int dq = nthr / Bg, dr = nthr - dq * Bg;
    constexpr int kPro = 8;                  // ring loads in flight per thread
    int m = tid / Bg, jl = tid - m * Bg;
    while (m < scan) {
      long long v[kPro];
      int mu[kPro], ju[kPro];
#pragma unroll
      for (int u = 0; u < kPro; ++u) {
        mu[u] = m;
        ju[u] = jl;
        v[u] = (m < scan) ? ld_dev(p.ring + (size_t)((rs0 + m) & kRingMask) * p.ring_stride + j0 + jl) : 0ll;
        jl += dr;
        m += dq;
        if (jl >= Bg) { jl -= Bg; ++m; }
      }
#pragma unroll
      for (int u = 0; u < kPro; ++u) {
        const int mm = mu[u], jj = ju[u];
        if (mm >= scan) break;
        const int rs = (rs0 + mm) & kRingMask;
        if (mm < take) {
          acc[(size_t)(sl0 + mm >= DL ? sl0 + mm - DL : sl0 + mm) * a.B + jj] = v[u];
          if (v[u] != 0) st_dev(p.ring + (size_t)rs * p.ring_stride + j0 + jj, 0ll);
        } else if (mm >= DL && v[u] != 0) {
          atomicOr(&fbits[rs * a.BW + (jj >> 5)], 1u << (jj & 31));
        }
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();                            // the window is in LDS before step n0's input is read
  for (int it = 0; it < steps; ++it) {
    const long long n = n0 + it;
    const bool timing = kTime && tid == 0;
    long long tp0 = timing ? wall_clock64() : 0;
    const int sn1 = (sn + 1 == DL) ? 0 : sn + 1;
    const int snm2 = (sn >= 2) ? sn - 2 : sn - 2 + DL;   // slot of step n-2
    const int par = (int)(n & 1);
    const size_t rslot = (size_t)(n & (kRecSlots - 1));  // record slot of step n
    // ---- rest of the update of step n (its input into I), spike decision of
    //      step n+1 ------------------------------------------------------------
    if (updw) {
      absorb(n, sn);
      int spiked = 0;
      if (it + 1 < steps) spiked = decide(n + 1);
      if (timing) { const long long t = wall_clock64(); ph[0] += t - tp0; tp0 = t; }
      // ---- record of step n+1 -------------------------------------------------
      if (it + 1 < steps) publish(n + 1, spiked, next16(t16n));
      if (timing) { const long long t = wall_clock64(); ph[1] += t - tp0; tp0 = t; }
      // drive of step n+1
      if (upd && it + 1 < steps) kdrive = (int)((drive_counts(n + 1, qlocal, seed, qpops, s_table) >> (8 * qk)) & 0xFFu);
    }
    const unsigned long long tag16 = (unsigned long long)t16n << 48;
    // ---- while the records of step n arrive: polling (the last wavefront,
    //      from the top of the step unless it holds targets); the pipelined
    //      delivery (block bounds of step n-1, entries of step n-2) in items
    //      claimed by the other wavefronts, those without targets from the top
    const long long tp_wait = kTime ? wall_clock64() : 0;
    if (pollw) {
      const int lane = tid & 63;
      if (lane == 0) { s_nids = 0; s_nbig = 0; }   // read after the previous wait
      long long t_poll = 0;          // the wall clock is read every 256 rounds only
      unsigned spins = 0;
      unsigned todo = 0;
#pragma unroll
      for (int r = 0; r < kPoll; ++r)
        if (lane + 64 * r < a.G) todo |= 1u << r;
      while (todo) {
        unsigned long long w0[kPoll];
#pragma unroll
        for (int r = 0; r < kPoll; ++r)
          w0[r] = ((todo >> r) & 1u) ? ld_dev(&a.flags[((size_t)(lane + 64 * r) * kRecSlots + rslot) * kPersistFlagStride])
                                     : 0ull;
#pragma unroll
        for (int r = 0; r < kPoll; ++r) {
          if (!((todo >> r) & 1u) || (w0[r] & 0xFFFF000000000000ull) != tag16) continue;
          const int h = lane + 64 * r;
          const int c = (int)((w0[r] >> 36) & 0x3FFu);
          // words 1.. for spikes 5..39 (one round trip for them, then their tags)
          constexpr int kMoreWords = kPersistFlagStride - 1;
          unsigned long long wk[kMoreWords];
          const int nwk = (c > kW0Ids) ? (min(c, kInline) - kW0Ids + kWIds - 1) / kWIds : 0;
          bool ok = true;
          if (nwk > 0) {
            const unsigned long long* rec = a.flags + ((size_t)h * kRecSlots + rslot) * kPersistFlagStride;
#pragma unroll
            for (int k = 0; k < kMoreWords; ++k) wk[k] = (k < nwk) ? ld_dev(&rec[1 + k]) : 0ull;
#pragma unroll
            for (int k = 0; k < kMoreWords; ++k)
              if (k < nwk) ok &= ((wk[k] & 0xFFFF000000000000ull) == tag16);
          }
          if (!ok) continue;
          s_cnt[h] = c;
          // the step's id list in arrival order (the order of integer sums
          // does not matter); ids beyond the 39th are fetched after the wait
          if (c > 0) {
            const int o = atomicAdd(&s_nids, c);
            const int ci = min(c, kInline);
            for (int k = 0; k < ci; ++k) {
              if (o + k >= kListCap) break;
              const unsigned long long wv = (k < kW0Ids) ? w0[r] : wk[(k - kW0Ids) / kWIds];
              const int f = (k < kW0Ids) ? k : (k - kW0Ids) % kWIds;
              s_ids[par * kListCap + o + k] = pbs[r] + (int)((wv >> (9 * f)) & 0x1FFu);
            }
            if (c > kInline) {
              const int b = atomicAdd(&s_nbig, 1);
              if (b < kBigCap) s_big[b] = make_int2(h, o);
            }
          }
          todo &= ~(1u << r);
        }
        // the ids listed so far are complete records (a busy producer's
        // later ids come after the wait, so the count stops advancing there)
        if (lane == 0 && s_nbig == 0 && s_nids <= list_cap)
          __hip_atomic_store(&s_nready, s_nids, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (!todo) break;
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255u) == 0u && (t_poll == 0 ? ((t_poll = wall_clock64()), false) : wall_clock64() - t_poll > a.wait_ticks)) {
          atomicOr(p.overflow, 2u);
          s_abort = 1;
#pragma unroll
          for (int r = 0; r < kPoll; ++r)
            if ((todo >> r) & 1u) s_cnt[lane + 64 * r] = 0;
          break;
        }
      }
      if (lane == 0) __hip_atomic_store(&s_polldone, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (kTime && tid == nthr - 64) ph[6] += wall_clock64() - tp_wait;
    }
    if (!pollw || !overlap) {
      const int pn1 = par ^ 1, pn2 = par;  // parity of steps n-1 and n-2
      const int nb2 = (S2 + kItemSpikes - 1) / kItemSpikes, items = nb2 + ((S1 + 63) >> 6);
      const int lane = tid & 63;
      unsigned long long ev = 0;
      for (;;) {
        int i = 0;
        if (lane == 0) i = atomicAdd(&s_work, 1);
        i = __builtin_amdgcn_readfirstlane(i);
        if (i >= items) break;
        if (i < nb2) {                     // entries (delay >= 3) of kItemSpikes spikes of step n-2
          wave_entries(p, blk, kItemSpikes * i, min(S2, kItemSpikes * (i + 1)), n - 2, snm2, 3, bounds_of(pn2));
        } else {                           // block bounds of spikes 64(i - nb2).. of step n-1
          const int k = 64 * (i - nb2) + lane;
          if (k < S1) {
            const long long* bi = a.blk + (size_t)s_ids[pn1 * kListCap + k] * (a.G + 1) + g;
            const long long b0 = bi[0], b1 = bi[1];
            s_lo[pn1 * kListCap + k] = b0;
            s_len[pn1 * kListCap + k] = (int)(b1 - b0);
            ev += (unsigned long long)(b1 - b0);
          }
        }
      }
      if (ev) atomicAdd(&s_events, ev);
      // the last wavefront without targets, its items done, adds the near
      // events of the first ids listed (at most kEarlyNear) while the poll
      // goes on
      if (overlap && wave == nw - 2 && !updw) {
        int done = 0;
        for (;;) {
          const int pd = __hip_atomic_load(&s_polldone, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
          const int ready = __hip_atomic_load(&s_nready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
          const int upto = min(ready, kEarlyNear);
          if (upto > done) {
            wave_near(a, blk, s_ids + par * kListCap, done, upto, gpos, sn1, sn1 + 1 == DL ? 0 : sn1 + 1);
            done = upto;
            continue;
          }
          if (done >= kEarlyNear || pd) break;
          __builtin_amdgcn_s_sleep(1);
        }
        if (lane == 0) s_ndone = done;
      }
      if (timing) ph[5] += wall_clock64() - tp_wait;
    }
    __syncthreads();                       // s_cnt, the inline ids and the poller's list complete
    const int ndone = s_ndone;             // ids whose near events are in already
    if (tid == 0) { s_work = 0; s_nready = 0; s_polldone = 0; }   // untouched until the next step (barriers below)
    if (s_abort) break;
    int S = s_nids;
    int* ids_n = s_ids + par * kListCap;
    if (S <= list_cap && s_nbig <= kBigCap) {
      // ---- the spikes of step n are listed: fetch the ids beyond the
      //      39th of busy producers, then each wavefront delivers the near
      //      events of its share of the ids not delivered during the poll ---
      if (timing) { const long long t = wall_clock64(); ph[2] += t - tp0; tp0 = t; }
      const int nbig = s_nbig;
      if (nbig > 0) {
        for (int e = 0; e < nbig; ++e) {
          const int h = s_big[e].x, o = s_big[e].y, c = s_cnt[h];
          for (int k = kInline + tid; k < c; k += nthr) ids_n[o + k] = ld_dev(&a.pub[((size_t)h * kRecSlots + rslot) * a.B + k]);
        }
        __syncthreads();
      }
      const int k0 = ndone + (int)((long long)(S - ndone) * wave / nw), k1 = ndone + (int)((long long)(S - ndone) * (wave + 1) / nw);
      if (timing) { const long long t = wall_clock64(); ph[3] += t - tp0; tp0 = t; }
      wave_near(a, blk, ids_n, k0, k1, gpos, sn1, sn1 + 1 == DL ? 0 : sn1 + 1);
      __syncthreads();
      if (timing) { const long long t = wall_clock64(); ph[4] += t - tp0; tp0 = t; }
      S2 = S1;
      S1 = S;
      sn = sn1;
      t16n = next16(t16n);
      continue;
    }
    // ---- more spikes than the list holds: listing by producer order
    //      (count scan), then every event of the step delivered at once ----
    if (ndone > 0) {   // the early near events come out again (exact integer sums), the listing overwrites their ids
      const int k0 = (int)((long long)ndone * wave / nw), k1 = (int)((long long)ndone * (wave + 1) / nw);
      wave_near(a, blk, ids_n, k0, k1, gpos, sn1, sn1 + 1 == DL ? 0 : sn1 + 1, -1);
      __syncthreads();
    }
    // thread t sums producers 2t and 2t+1 (G <= 2 * threads)
    const int c0 = (2 * tid < a.G) ? s_cnt[2 * tid] : 0;
    const int c1 = (2 * tid + 1 < a.G) ? s_cnt[2 * tid + 1] : 0;
    const int pre_h = block_exscan(c0 + c1, s_tmp[1], &S);   // also a barrier
    if (2 * tid < a.G) s_pre[2 * tid] = pre_h;
    if (2 * tid + 1 < a.G) s_pre[2 * tid + 1] = pre_h + c0;
    if (tid == 0) s_pre[a.G] = S;
    __syncthreads();
    if (timing) { const long long t = wall_clock64(); ph[2] += t - tp0; tp0 = t; }
    for (int base = 0; base < S; base += kListCap) {
      const int cnt = min(kListCap, S - base);
      const int k0 = (int)((long long)cnt * wave / nw), k1 = (int)((long long)cnt * (wave + 1) / nw);
      for (int k = k0 + (tid & 63); k < k1; k += 64) {
        const int gk = base + k;
        int lo = 0, hi = a.G;                 // producer h: s_pre[h] <= gk < s_pre[h+1]
        while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (s_pre[mid] <= gk) lo = mid; else hi = mid; }
        const int kk = gk - s_pre[lo];
        if (kk < kInline) {                   // from the producer's record word (still this step's)
          const int wi = (kk < kW0Ids) ? 0 : 1 + (kk - kW0Ids) / kWIds;
          const int f = (kk < kW0Ids) ? kk : (kk - kW0Ids) % kWIds;
          const unsigned long long wv = ld_dev(&a.flags[((size_t)lo * kRecSlots + rslot) * kPersistFlagStride + wi]);
          ids_n[k] = a.bstart[lo] + (int)((wv >> (9 * f)) & 0x1FFu);
        } else {
          ids_n[k] = ld_dev(&a.pub[((size_t)lo * kRecSlots + rslot) * a.B + kk]);
        }
      }
      if (timing) { const long long t = wall_clock64(); ph[3] += t - tp0; tp0 = t; }
      if (S <= kListCap) {
        wave_near(a, blk, ids_n, k0, k1, gpos, sn1, sn1 + 1 == DL ? 0 : sn1 + 1);   // reads the ids this wavefront wrote
      } else {
        // too many spikes to keep: deliver all events of this chunk now
        unsigned long long ev = 0;
        auto direct = [&](int k, long long* lo, int* len) {
          const long long* bi = a.blk + (size_t)ids_n[k] * (a.G + 1) + g;
          *lo = bi[0];
          *len = (int)(bi[1] - *lo);
          ev += (unsigned long long)*len;
        };
        wave_entries(p, blk, k0, k1, n, sn, 1, direct);
        if (ev) atomicAdd(&s_events, ev);
      }
      __syncthreads();
      if (timing) { const long long t = wall_clock64(); ph[4] += t - tp0; tp0 = t; }
    }
    S2 = S1;
    S1 = (S <= kListCap) ? S : 0;
    sn = sn1;
    t16n = next16(t16n);
  }
  // ---- pipelined events still due: entries of step n_end-2, bounds and
  //      entries of step n_end-1 --------------------------------------------
  const long long n_end = n0 + steps;
  if (!s_abort && steps > 0) {
    const int pl = (int)((n_end - 1) & 1), pl2 = pl ^ 1;
    const int sl = (sn == 0) ? DL - 1 : sn - 1;          // slot of step n_end-1
    const int sl2 = (sl == 0) ? DL - 1 : sl - 1;         // slot of step n_end-2
    if (S2 > 0) {
      const int k0 = (int)((long long)S2 * wave / nw), k1 = (int)((long long)S2 * (wave + 1) / nw);
      wave_entries(p, blk, k0, k1, n_end - 2, sl2, 3, bounds_of(pl2));
    }
    if (S1 > 0) {
      const int k0 = (int)((long long)S1 * wave / nw), k1 = (int)((long long)S1 * (wave + 1) / nw);
      unsigned long long ev = 0;
      const int* ids_l = s_ids + pl * kListCap;
      auto direct = [&](int k, long long* lo, int* len) {
        const long long* bi = a.blk + (size_t)ids_l[k] * (a.G + 1) + g;
        *lo = bi[0];
        *len = (int)(bi[1] - *lo);
        ev += (unsigned long long)*len;
      };
      wave_entries(p, blk, k0, k1, n_end - 1, sl, 3, direct);
      if (ev) atomicAdd(&s_events, ev);
    }
  }
  __syncthreads();
  // ---- epilogue: state, counters, LDS window back into the global ring ------
  if (upd) { p.y[j0 + tid] = y; p.I[j0 + tid] = I; p.r[j0 + tid] = r; }
  if (tid < p.n_pops) p.wg_spikes[(size_t)g * p.n_pops + tid] += s_popcnt[tid];
  if (kTime && tid == 0) {
    for (int k = 0; k < 6; ++k) a.phase[(size_t)g * 8 + k] += (unsigned long long)ph[k];
    a.phase[(size_t)g * 8 + 7] += (unsigned long long)steps;
  }
  if (kTime && tid == nthr - 64) a.phase[(size_t)g * 8 + 6] += (unsigned long long)ph[6];
  if (tid == 0) {
    p.raster_cnt[g] = rcnt;
    p.wg_events[g] += s_events;
  }
  // the global entry of a window slot is zero unless far events were added
  // to it (its far bit): a store, else an add.  (m, jl) stepped as in the prologue.
  if (Bg > 0) {
    const int sl0 = (int)(n_end % DL), rs0 = (int)(n_end & kRingMask);
    const int dq = nthr / Bg, dr = nthr - dq * Bg;
    int m = tid / Bg, jl = tid - m * Bg;
    while (m < DL) {
      const long long v = acc[(size_t)(sl0 + m >= DL ? sl0 + m - DL : sl0 + m) * a.B + jl];
      if (v != 0) {
        const int rs = (rs0 + m) & kRingMask;
        long long* e = p.ring + (size_t)rs * p.ring_stride + j0 + jl;
        if (fbits[rs * a.BW + (jl >> 5)] & (1u << (jl & 31)))
          atomicAdd(reinterpret_cast<unsigned long long*>(e), (unsigned long long)v);
        else
          st_dev(e, v);
      }
      jl += dr;
      m += dq;
      if (jl >= Bg) { jl -= Bg; ++m; }
    }
  }
  // The last workgroup to finish (every other one has read all the records it
  // will read) clears the spike records for the next launch and advances the
  // step counter (every workgroup read it before its first record).
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    unsigned long long* done = a.flags + persist_record_words(a.G);
    s_last = (__hip_atomic_fetch_add(done, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (unsigned long long)(a.G - 1));
  }
  __syncthreads();
  if (s_last) {
    const int words = (int)persist_record_words(a.G);
    for (int k = tid; k < words; k += nthr) st_dev(&a.flags[k], 0ull);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) {
      st_dev(p.step_base, n_end);
      __hip_atomic_store(a.flags + persist_record_words(a.G), 0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The exchange of k_persist with nothing else: every step, each of the G
// workgroups publishes a step-tagged record (word 0 as in k_persist, no
// spikes) and its last wavefront polls all G records of the step the same
// way (four or eight producers per lane, device-scope loads, a short sleep between
// rounds); then a barrier and the next step.  The time per step is the floor
// the persistent kernel's step cannot go below.  Records are cleared by the
// last workgroup to finish, as in k_persist.
template <int kPoll>
__global__ __launch_bounds__(kPersistMaxBlock) void k_exchange_probe(unsigned long long* flags, int G, long long steps,
                                                                     long long wait_ticks, unsigned* err) {
  __shared__ int s_abort, s_last;
  const int g = blockIdx.x, tid = threadIdx.x, nthr = blockDim.x;
  const int nw = nthr >> 6, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) s_abort = 0;
  __syncthreads();
  for (long long n = 0; n < steps; ++n) {
    const unsigned long long tag16 = (unsigned long long)((n + 1) % 65535 + 1) << 48;
    const size_t rslot = (size_t)(n % kRecSlots);
    if (tid == 0) st_dev(&flags[((size_t)g * kRecSlots + rslot) * kPersistFlagStride], tag16);
    if (wave == nw - 1) {
      long long t_poll = 0;          // the wall clock is read every 256 rounds only
      unsigned spins = 0;
      unsigned todo = 0;
#pragma unroll
      for (int r = 0; r < kPoll; ++r)
        if (lane + 64 * r < G) todo |= 1u << r;
      while (todo) {
        unsigned long long w0[kPoll];
#pragma unroll
        for (int r = 0; r < kPoll; ++r)
          w0[r] = ((todo >> r) & 1u) ? ld_dev(&flags[((size_t)(lane + 64 * r) * kRecSlots + rslot) * kPersistFlagStride])
                                     : 0ull;
#pragma unroll
        for (int r = 0; r < kPoll; ++r)
          if (((todo >> r) & 1u) && (w0[r] & 0xFFFF000000000000ull) == tag16) todo &= ~(1u << r);
        if (!todo) break;
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255u) == 0u && (t_poll == 0 ? ((t_poll = wall_clock64()), false) : wall_clock64() - t_poll > wait_ticks)) {
          atomicOr(err, 2u);
          s_abort = 1;
          break;
        }
      }
    }
    __syncthreads();
    if (s_abort) break;
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (tid == 0) {
    unsigned long long* done = flags + persist_record_words(G);
    s_last = (__hip_atomic_fetch_add(done, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == (unsigned long long)(G - 1));
  }
  __syncthreads();
  if (s_last) {
    const int words = (int)persist_record_words(G);
    for (int k = tid; k < words; k += nthr) st_dev(&flags[k], 0ull);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) __hip_atomic_store(flags + persist_record_words(G), 0ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

hipError_t launch_exchange_probe(unsigned long long* flags, int G, int block, long long steps, long long wait_ticks,
                                 unsigned* err, hipStream_t s) {
  if (G < 1 || G > kPersistMaxBlock || block < 64 || block > kPersistMaxBlock || block % 64) return hipErrorInvalidValue;
  if (G <= 256)
    hipLaunchKernelGGL(k_exchange_probe<4>, dim3(G), dim3(block), 0, s, flags, G, steps, wait_ticks, err);
  else
    hipLaunchKernelGGL(k_exchange_probe<8>, dim3(G), dim3(block), 0, s, flags, G, steps, wait_ticks, err);
  return hipGetLastError();
}

// blk[i][g] = first synapse of row i whose target is >= bstart[g] (rows sorted by target).
__global__ void k_build_blk(const int64_t* row_ptr, const int32_t* tgt, long long n_pad, int G, const int* bstart,
                            long long* blk) {
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= n_pad * (G + 1)) return;
  const long long i = idx / (G + 1);
  const int g = (int)(idx - i * (G + 1));
  long long lo = row_ptr[i], hi = row_ptr[i + 1];
  const long long key = bstart[g];
  while (lo < hi) { const long long mid = (lo + hi) >> 1; if (tgt[mid] < key) lo = mid + 1; else hi = mid; }
  blk[idx] = lo;
}

// Range of row i with targets in [t0, t1) (rows sorted by target).
__device__ __forceinline__ void row_range(const int64_t* row_ptr, const int32_t* tgt, long long i, long long t0,
                                          long long t1, long long* b, long long* e) {
  long long lo = row_ptr[i], hi = row_ptr[i + 1];
  while (lo < hi) { const long long mid = (lo + hi) >> 1; if (tgt[mid] < t0) lo = mid + 1; else hi = mid; }
  *b = lo;
  hi = row_ptr[i + 1];
  while (lo < hi) { const long long mid = (lo + hi) >> 1; if (tgt[mid] < t1) lo = mid + 1; else hi = mid; }
  *e = lo;
}

// Near (delay 1-2) synapses of row i that land in the block of the workgroup
// at XCD-order position p: counts into cnt[i][p] (p < G; cnt[i][G] = 0 for
// the exclusive scan).
__global__ void k_near_count(const int32_t* tgt, const uint8_t* dly, const long long* blk, long long n_pad, int G,
                             unsigned* cnt) {
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= n_pad * (G + 1)) return;
  const long long i = idx / (G + 1);
  const int pos = (int)(idx - i * (G + 1));
  unsigned c = 0;
  if (pos < G) {
    const long long* b = blk + i * (G + 1) + xcd_wg(pos, G);
    for (long long k = b[0]; k < b[1]; ++k) c += (dly[k] <= 2);
  }
  cnt[idx] = c;
}

// Entries at nb[i][p]...: (delay-2 flag | target - bstart[g]) << 32 | weight,
// in row order, for the workgroup g at position p.
__global__ void k_near_fill(const int32_t* tgt, const int32_t* wq, const uint8_t* dly, const long long* blk,
                            const int* bstart, long long n_pad, int G, const unsigned* nb, unsigned long long* ne) {
  const long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (idx >= n_pad * (G + 1)) return;
  const long long i = idx / (G + 1);
  const int pos = (int)(idx - i * (G + 1));
  if (pos == G) return;
  const int g = xcd_wg(pos, G);
  const long long* b = blk + i * (G + 1) + g;
  unsigned o = nb[idx];
  for (long long k = b[0]; k < b[1]; ++k)
    if (dly[k] <= 2)
      ne[o++] = ((unsigned long long)((unsigned)(tgt[k] - bstart[g]) | (dly[k] == 2 ? kNearD2 : 0u)) << 32) |
                (unsigned)wq[k];
}

size_t persist_lds_bytes(int G, int B, int DL) {
  const int BW = (B + 31) / 32;
  size_t b = (size_t)DL * B * 8 + (size_t)128 * BW * 4 + (size_t)(G + 1) * 4 +
             (size_t)kListCap * 4 * 4;
  b = (b + 15) & ~(size_t)15;
  return b + (size_t)2 * kListCap * 8;
}

// The instances of k_persist (recording, timing, poll width); shapes are
// checked against all of them.
const void* const kPersistFns[8] = {
    (const void*)k_persist<false, false, 4>, (const void*)k_persist<true, false, 4>,
    (const void*)k_persist<false, true, 4>,  (const void*)k_persist<true, true, 4>,
    (const void*)k_persist<false, false, 8>, (const void*)k_persist<true, false, 8>,
    (const void*)k_persist<false, true, 8>,  (const void*)k_persist<true, true, 8>};

hipError_t persist_static_lds(size_t* bytes) {
  *bytes = 0;
  for (const void* f : kPersistFns) {
    hipFuncAttributes attr;
    const hipError_t e = hipFuncGetAttributes(&attr, f);
    if (e != hipSuccess) return e;
    *bytes = std::max<size_t>(*bytes, attr.sharedSizeBytes);
  }
  return hipSuccess;
}

hipError_t persist_occupancy(int block, size_t lds, int* blocks_per_cu) {
  *blocks_per_cu = 1 << 30;
  for (const void* f : kPersistFns) {
    int occ = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, f, block, lds);
    if (e != hipSuccess) return e;
    *blocks_per_cu = std::min(*blocks_per_cu, occ);
  }
  return hipSuccess;
}

template <bool kRec, bool kTime>
static void launch_persist_as(const DevNet& p, const PersistArgs& a, int steps, int block, size_t lds, hipStream_t s) {
  auto* const kf = (a.G <= 256) ? k_persist<kRec, kTime, 4> : k_persist<kRec, kTime, 8>;
  hipLaunchKernelGGL(kf, dim3(a.G), dim3(block), lds, s, p, a, steps);
}

hipError_t launch_persist(const DevNet& p, const PersistArgs& a, int steps, int block, hipStream_t s) {
  const size_t lds = persist_lds_bytes(a.G, a.B, a.DL);
  const bool rec = p.xrec != nullptr || p.ck_y != nullptr, tim = a.phase != nullptr;
  if (rec && tim) launch_persist_as<true, true>(p, a, steps, block, lds, s);
  else if (rec) launch_persist_as<true, false>(p, a, steps, block, lds, s);
  else if (tim) launch_persist_as<false, true>(p, a, steps, block, lds, s);
  else launch_persist_as<false, false>(p, a, steps, block, lds, s);
  return hipGetLastError();
}

hipError_t launch_build_blk(const int64_t* row_ptr, const int32_t* tgt, long long n_pad, int G, const int* bstart,
                            long long* blk, hipStream_t s) {
  const long long total = n_pad * (G + 1);
  hipLaunchKernelGGL(k_build_blk, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, row_ptr, tgt, n_pad, G, bstart,
                     blk);
  return hipGetLastError();
}

hipError_t launch_near_count(const int32_t* tgt, const uint8_t* dly, const long long* blk, long long n_pad, int G,
                             unsigned* cnt, hipStream_t s) {
  const long long total = n_pad * (G + 1);
  hipLaunchKernelGGL(k_near_count, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, tgt, dly, blk, n_pad, G, cnt);
  return hipGetLastError();
}

hipError_t launch_near_fill(const int32_t* tgt, const int32_t* wq, const uint8_t* dly, const long long* blk,
                            const int* bstart, long long n_pad, int G, const unsigned* nb, unsigned long long* ne,
                            hipStream_t s) {
  const long long total = n_pad * (G + 1);
  hipLaunchKernelGGL(k_near_fill, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, tgt, wq, dly, blk, bstart,
                     n_pad, G, nb, ne);
  return hipGetLastError();
}

hipError_t persist_set_lds_limit(size_t lds) {
  for (const void* f : kPersistFns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mc
