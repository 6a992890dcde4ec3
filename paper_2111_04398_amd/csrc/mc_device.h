// mc_device.h -- device-side data layout of libmc and kernel entry points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_common.h"

namespace mc {

// Everything a simulation kernel reads or writes, by value in the kernel
// argument buffer.  Neuron ids on the device are "padded" ids: every
// instance starts at a multiple of 4 so that one Philox block (four words)
// drives one aligned quad of neurons of a single instance.
struct DevNet {
  int64_t n_pad;            // padded neuron count (multiple of 4)
  int64_t n_quads;          // n_pad / 4
  int64_t ring_stride;      // elements per ring slot (>= n_pad, multiple of 64)
  int32_t n_pops;
  // synapse store (canonical order, padded ids)
  const int64_t* row_ptr;   // [n_pad+1]
  const int32_t* tgt;       // [M]
  const int32_t* wq;        // [M]
  const uint8_t* dly;       // [M]
  // state
  double* y;                // [n_pad] V - E_L
  double* I;                // [n_pad]
  int32_t* r;               // [n_pad] refractory steps left
  long long* ring;          // [kRingSlots][ring_stride] pending integer input (2^-16 pA)
  // per-quad drive metadata
  const uint64_t* qseed;    // [n_quads] instance seed
  const uint32_t* qlocal;   // [n_quads] quad index inside its instance
  const uint32_t* qpops;    // [n_quads] population of each of the 4 neurons (0xFF: padding)
  const uint64_t* table;    // [n_pops*64] Poisson inverse CDF
  // constants
  double P11, P21, P22, P20, i_e, theta, y_reset;
  long long jext_q;
  int32_t ref_steps;
  // step counter: kernels simulate step (*step_base + offset)
  long long* step_base;
  // recording: one private raster segment per workgroup
  int2* raster;             // [n_wg][raster_cap]
  long long raster_cap;
  long long* raster_cnt;    // [n_wg]
  unsigned long long* wg_events;   // [n_wg]
  unsigned long long* wg_spikes;   // [n_wg * n_pops]
  unsigned* overflow;       // set if a raster segment would overflow
  // adjoint forward: when xrec is set, the integer input (ring, far part
  // and the Poisson drive) of every neuron at step n in [xrec_step0,
  // xrec_step0 + xrec_steps) goes to xrec[(n - xrec_step0) * ring_stride + i]
  long long* xrec;
  long long xrec_step0;
  long long xrec_steps;
  // adjoint forward: when ck_y is set, the state (y, I, r) of every neuron
  // before the update of step ck_step0 + k * ck_every (k < ck_count) goes to
  // ck_*[k * ring_stride + i]
  double* ck_y;
  double* ck_I;
  int32_t* ck_r;
  long long ck_step0;
  long long ck_every;
  long long ck_count;
  // target-owner scheme: per-instance spike lists of the current step
  int32_t n_inst;
  const int32_t* qinst;     // [n_quads] instance of each quad
  const int64_t* inst_base; // [n_inst+1] first padded id of each instance
  int* ilist;               // [2][n_pad] spike ids by step parity, instance b at inst_base[b]
  int* icnt;                // [2][n_inst] list lengths by step parity
};

}  // namespace mc

namespace mc {

// Arguments of the persistent LDS kernel (target-owner delivery).
struct PersistArgs {
  int G;                       // workgroups (all co-resident, G <= 2 * block, G <= 512)
  int B;                       // most target neurons of one workgroup (multiple of 4, <= kPersistMaxB)
  const int* bstart;           // [G+1] workgroup g owns padded targets [bstart[g], bstart[g+1]) (multiples of 4)
  int DL;                      // near slots held in LDS (2..101)
  int horizon;                 // ring slots ahead of the first step that may hold input at launch (<= 127)
  int BW;                      // 32-bit words per far-bitmap row: ceil(B/32)
  const long long* blk;        // [n_pad][G+1] first synapse of each row with target >= bstart[g]
  unsigned long long* flags;   // [G][kRecSlots][8] spike records by step mod kRecSlots, then the
                               // launch's finish counter (one word, zero between launches)
  int* pub;                    // [G][kRecSlots][B] published spike ids beyond the seventh
  long long wait_ticks;        // longest wait for one step's records, in wall_clock64 ticks (then: error bit 2)
  unsigned long long* phase;   // optional [G*8]: summed wall_clock64 ticks per phase (nullptr: off)
  // near table: the delay-1/2 synapses of row i into workgroup g's block are
  // ne[nb[i][p] .. nb[i][p+1]) with p the position of g when the workgroups
  // are ordered by XCD (g mod 8, then g), each (target - bstart[g]) << 32 |
  // weight, bit 31 of the target field set for delay 2
  const unsigned* nb;          // [n_pad][G+1]
  const unsigned long long* ne;
  // spikes of a step above which it is listed in producer order after the
  // wait (0: the LDS list's capacity); a smaller value is a test hook that
  // sends ordinary steps down that path (phase-timing instance only)
  int list_cap;
};
constexpr int kPersistFlagStride = 8;
constexpr int kRecSlots = 4;            // spike records (and side arrays) per workgroup, by step mod 4
__host__ __device__ inline size_t persist_record_words(int G) { return (size_t)G * kRecSlots * kPersistFlagStride; }
__host__ __device__ inline size_t persist_flag_words(int G) { return persist_record_words(G) + kPersistFlagStride; }
constexpr int kPersistMaxB = 512;       // owned targets per workgroup (one per thread)
constexpr int kPersistMaxBlock = 512;   // threads per workgroup: 256 VGPRs per lane, no scratch spills
size_t persist_lds_bytes(int G, int B, int DL);
// Near table: counts per (source, workgroup), then (after an exclusive scan)
// the fill.
hipError_t launch_near_count(const int32_t* tgt, const uint8_t* dly, const long long* blk, long long n_pad, int G,
                             unsigned* cnt, hipStream_t s);
hipError_t launch_near_fill(const int32_t* tgt, const int32_t* wq, const uint8_t* dly, const long long* blk,
                            const int* bstart, long long n_pad, int G, const unsigned* nb, unsigned long long* ne,
                            hipStream_t s);
hipError_t persist_static_lds(size_t* bytes);
hipError_t persist_occupancy(int block, size_t lds, int* blocks_per_cu);
hipError_t persist_set_lds_limit(size_t lds);
hipError_t launch_persist(const DevNet& p, const PersistArgs& a, int steps, int block, hipStream_t s);
// Scratch of the allocation-free entry point (mc_noalloc.hip): spike records
// (noalloc_record_words() words, room for 512 workgroups) and the side array
// (512 x kRecSlots x 512 ints) of this device; and a record clear by kernel.
size_t noalloc_scratch_bytes();
size_t noalloc_record_words();
hipError_t noalloc_scratch(int device, unsigned long long** records, int** pub);
hipError_t launch_clear_records(unsigned long long* records, size_t words, hipStream_t s);
hipError_t launch_build_blk(const int64_t* row_ptr, const int32_t* tgt, long long n_pad, int G, const int* bstart,
                            long long* blk, hipStream_t s);

constexpr int kReplayChunkHost = 256;     // must equal the replay kernel's chunk
hipError_t launch_replay(const int2* spikes, const long long* first_item, int n_spikes, long long n_items,
                         const int64_t* row_ptr, const int32_t* tgt, const int32_t* wq, const uint8_t* dly,
                         long long* ring, long long stride, long long step0, int grid, hipStream_t s);
hipError_t launch_atomic_rate(unsigned long long* table, long long n, long long per_thread, int grid, hipStream_t s);
hipError_t launch_stream_read(const void* src, long long bytes, unsigned long long* sink, int grid, hipStream_t s);
hipError_t launch_atomic_slots(unsigned long long* table, long long slots, long long stride, long long n_targets,
                               long long n_items, int pattern, int gap, const unsigned char* dq, int grid,
                               hipStream_t s);
// Empty persistent loop of G co-resident workgroups exchanging one spike
// record per step (no neurons, no delivery): the exchange's latency floor.
// flags: persist_flag_words(G) words, zero on entry and on exit.
hipError_t launch_exchange_probe(unsigned long long* flags, int G, int block, long long steps, long long wait_ticks,
                                 unsigned* err, hipStream_t s);

// One segment of the adjoint's reverse pass (see mc_adjoint.hip).
struct AdjSeg {
  long long a;             // first step of the segment
  int len;                 // steps in the segment
  int R;                   // LI ring slots (power of two, >= len + 101)
  double c;                // 2 / (N S)
  double ystar;            // y* = V* - E_L
  const double* ck_y;      // checkpoint state at step a
  const double* ck_I;
  const int32_t* ck_r;
  const long long* xseg;   // [len][ring_stride] integer input, with the drive if x_has_drive, else without
  int x_has_drive;         // 1: xseg is the forward's full input record (no drive to redraw)
  double* rec_y;           // [len][ring_stride] post-step y
  uint8_t* rec_t;          // [len][ring_stride] step type
  double* li_ring;         // [R][ring_stride] LI(m) at slot m & (R-1)
  double* carry_ly;        // [ring_stride] Ly at step a+len on entry, at step a on exit
  double* carry_li;        // [ring_stride] LI likewise
  double* loss_part;       // [ring_stride] per-neuron sum of squared deviations
  unsigned long long* spike_count;   // recomputed spikes of this segment (added to)
};
constexpr int kGatherChunkHost = 256;     // must equal the gather kernel's chunk
hipError_t launch_adj_seed(long long* xseg, const long long* ring_ckpt, long long stride, long long a, int rows,
                           hipStream_t s);
hipError_t launch_adj_segment(const DevNet& p, const AdjSeg& a, hipStream_t s);
hipError_t launch_adj_verify(const int2* spikes, int n, const uint8_t* rec_t, long long stride, long long a,
                             unsigned* mismatch, hipStream_t s);
hipError_t launch_adj_gather(const int4* srcs, const long long* first, int nsrc, long long n_items, const int* times,
                             const int64_t* row_ptr, const int32_t* tgt, const uint8_t* dly, const double* li_ring,
                             long long stride, int R, long long last_m, void* grad, bool fp32, int grid, hipStream_t s);

// Persistent kernel with target-owner delivery into per-workgroup delay
// buckets (mc_bucket.hip).  Workgroup g owns padded targets [bt0[g],
// bt0[g+1]) of instance binst[g] (its blb[g]-th block; the instance's blocks
// are ifb[b] .. ifb[b+1]-1, the last instance's end at G); sub-rows as in
// OwnerArgs (boff, blk2).
struct BucketArgs {
  int G;                       // workgroups (all co-resident)
  int B;                       // most targets of one workgroup (multiple of 4, <= kBucketMaxB)
  const int* bt0;              // [G+1]
  const int* binst;            // [G]
  const int* blb;              // [G]
  const int* ifb;              // [n_inst]
  const int64_t* boff;         // [n_pad+1]
  const int32_t* blk2;
  unsigned long long* flags;   // persist_flag_words(G): spike records [G][kRecSlots][8], then the finish counter
  int* pub;                    // [G][kRecSlots][B] published ids beyond the record's
  unsigned long long* bk;      // [G][128][cap] bucket entries (local target << 32 | weight)
  int cap;                     // entries per bucket (more: device atomics into the ring)
  long long wait_ticks;        // longest wait for one step's records (wall_clock64 ticks)
  int horizon;                 // ring slots ahead of the first step that may hold input at launch
  unsigned long long* phase;   // optional [G*8]: summed wall_clock64 ticks per phase (nullptr: off)
  int inst_wg_max;             // most workgroups of one instance (<= 64: one producer polled per lane)
};
constexpr int kBucketMaxProducers = 512;   // workgroups of one instance
constexpr int kBucketMaxBlock = 512;       // threads per workgroup
constexpr int kBucketMaxB = 4092;          // targets per workgroup (12-bit local indices and count in the records)
hipError_t launch_bucket(const DevNet& p, const BucketArgs& a, int steps, int block, hipStream_t s);
// co-resident workgroups per CU of the instances launched when no instance
// has more than inst_wg_max workgroups
hipError_t bucket_occupancy(int B, int block, int inst_wg_max, int* blocks_per_cu);
hipError_t bucket_set_lds_limit(size_t lds);
__host__ __device__ size_t bucket_sum_slots(int B);
size_t bucket_lds_bytes(int B);

// Target-owner delivery (one kernel per step after the update kernel):
// block k owns padded targets [bt0[k], bt0[k+1]) of instance binst[k]; it is
// the lb = blb[k]-th block of that instance.  Row i's sub-row for the
// instance's block lb is [row_ptr[i] + blk2[boff[i] + lb], row_ptr[i] +
// blk2[boff[i] + lb + 1]).
struct OwnerArgs {
  int n_blocks;
  int bmax;                 // most targets of one block
  const int* bt0;           // [n_blocks+1]
  const int* binst;         // [n_blocks]
  const int* blb;           // [n_blocks]
  const int64_t* boff;      // [n_pad+1]
  const int32_t* blk2;      // [boff[n_pad]] offsets inside the row
};
constexpr int kOwnerBlock = 256;          // threads of the owner kernel
constexpr int kOwnerMaxTargets = 1024;    // targets of one owner block
hipError_t launch_step_lists(const DevNet& p, int offset, int qpw, int n_wg, int block, hipStream_t s);
hipError_t launch_owner(const DevNet& p, const OwnerArgs& a, int offset, hipStream_t s);
hipError_t launch_zero_lists(int* icnt, int n, hipStream_t s);
hipError_t launch_build_blk2(const int64_t* row_ptr, const int32_t* tgt, long long n_pad, const int64_t* boff,
                             const int32_t* qinst, const int* inst_first_block, const int* bt0, int32_t* blk2,
                             hipStream_t s);

constexpr int kMaxQuadsPerWgHost = 256;   // must equal the kernel's per-workgroup quad limit
// wave_rows: 0 = every thread of the workgroup walks each spiking row in
// turn; 1 = each wavefront walks whole rows (spikes dealt round robin).
hipError_t launch_step(const DevNet& p, int offset, int qpw, int n_wg, int block, int wave_rows, hipStream_t s);
hipError_t launch_advance(long long* step_base, int steps, hipStream_t s);
hipError_t launch_inject(long long* ring, long long idx, long long value, hipStream_t s);
// New weights (mode 0: set from pA values; 1/2: one gradient step with a
// double/float gradient and rate eta); check pass sets *bad, else writes.
hipError_t launch_weights(int32_t* wq, const void* src, int mode, double eta, long long M, unsigned* bad, bool check,
                          hipStream_t s);
// Connections of the Bernoulli rule drawn on the device (the host builder's
// ConnBuilder; grid: workgroups of 256 threads; s: the stream it uses).
struct ConnBuilder;
ConnBuilder* new_device_conn(int grid, hipStream_t s);
// Raster segments' used prefixes -> one contiguous array (off: [n_seg+1] exclusive prefix of the counts).
hipError_t launch_raster_pack(const int2* raster, long long cap, const long long* off, int n_seg, int2* out,
                              hipStream_t s);
}  // namespace mc
