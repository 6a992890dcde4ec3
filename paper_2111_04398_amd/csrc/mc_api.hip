// mc_api.hip -- the C interface of libmc (include/mc.h): handle management,
// device memory plan, graph-replayed simulation loop, spike export,
// introspection and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "mc.h"
#include "mc_build.h"
#include "mc_device.h"

using namespace mc;

namespace {

thread_local std::string g_last_error;

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// On failure the runtime's last-error state is read and cleared as well, so
// that a later launch check does not report this failure again.
#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e__ = (expr);                                                               \
    if (e__ != hipSuccess) {                                                               \
      (void)hipGetLastError();                                                             \
      return set_error(e__ == hipErrorOutOfMemory ? MC_ERR_OOM : MC_ERR_HIP,               \
                       std::string(#expr) + ": " + hipGetErrorString(e__));                \
    }                                                                                      \
  } while (0)

inline int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

// Longest wait of a persistent workgroup for one step's spike records before
// the kernel gives up (error bit 2): a step takes microseconds, so seconds
// mean a workgroup that never publishes.
constexpr long long kWaitSeconds = 5;

// Entries per delay bucket of the bucket scheme (a full bucket sends further
// events of that arrival step to the ring with device atomics).
constexpr int kBucketCap = 8192;

// Error bits the kernels set in the overflow word.
constexpr unsigned kErrRasterOverflow = 1u, kErrWaitTimeout = 2u;

// Device memory of a network: from the caller's allocator hooks if the
// configuration gives them (e.g. a framework's caching allocator), else
// hipMalloc / hipFree.
struct Alloc {
  void* (*fn)(size_t, void*) = nullptr;
  void (*fr)(void*, void*) = nullptr;
  void* ctx = nullptr;
};

template <class T>
int dev_alloc(const Alloc& A, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  const size_t bytes = count * sizeof(T);
  if (A.fn) {
    *p = static_cast<T*>(A.fn(bytes, A.ctx));
    if (!*p) return set_error(MC_ERR_OOM, "the allocator hook returned NULL for " + std::to_string(bytes) + " bytes");
    if (reinterpret_cast<uintptr_t>(*p) % 256) {
      A.fr(*p, A.ctx);
      *p = nullptr;
      return set_error(MC_ERR_INVALID_ARG, "the allocator hook returned memory not aligned to 256 bytes");
    }
    return MC_OK;
  }
  hipError_t e = hipMalloc((void**)p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();   // the runtime keeps the failure as its last error: the next launch check would see it
    return set_error(e == hipErrorOutOfMemory ? MC_ERR_OOM : MC_ERR_HIP,
                     std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
  }
  return MC_OK;
}

template <class T>
void dev_free(const Alloc& A, T*& p) {
  if (p) {
    if (A.fr) A.fr((void*)p, A.ctx);
    else (void)hipFree((void*)p);
  }
  p = nullptr;
}

// Device buffers of one adjoint call, freed on every exit path.
struct AdjBuffers {
  const Alloc& A;
  std::vector<void*> ptrs;
  explicit AdjBuffers(const Alloc& a) : A(a) {}
  template <class T>
  int alloc(T** p, size_t count) {
    int rc = dev_alloc(A, p, count);
    if (rc == MC_OK) ptrs.push_back((void*)*p);
    return rc;
  }
  ~AdjBuffers() {
    for (void* p : ptrs) dev_free(A, p);
  }
};

}  // namespace

struct mc_net {
  HostNet h;
  Alloc alloc;                         // device memory of this network
  bool host_only = false;
  bool failed = false;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // padded layout
  int64_t n_pad = 0, n_quads = 0, ring_stride = 0;
  std::vector<int64_t> inst_off_pad;
  // device store and state
  int64_t* d_row_ptr = nullptr;
  int32_t* d_tgt = nullptr;
  int32_t* d_wq = nullptr;
  uint8_t* d_dly = nullptr;
  double* d_y = nullptr;
  double* d_I = nullptr;
  int32_t* d_r = nullptr;
  long long* d_ring = nullptr;
  uint64_t* d_qseed = nullptr;
  uint32_t* d_qlocal = nullptr;
  uint32_t* d_qpops = nullptr;
  uint64_t* d_table = nullptr;
  long long* d_step = nullptr;
  // persistent LDS scheme
  int n_cu = 0;
  int wall_khz = 100000;               // wall_clock64 rate (kHz)
  int lds_max = 65536;
  int pG = 0, pB = 0, pDL = 0;
  int horizon = kRingSlots - 1;        // ring slots ahead of the current step that may hold input
  long long* d_blk = nullptr;
  unsigned long long* d_flags = nullptr;
  unsigned long long* d_bk = nullptr;  // bucket scheme: [G][128][bk_cap] entries
  int bk_cap = 0;
  int* d_pub = nullptr;
  int* d_bstart = nullptr;
  std::vector<int> bstart_host;        // [pG+1] target blocks of the persistent workgroups
  // target-owner scheme
  int32_t* d_qinst = nullptr;          // [n_quads]
  int64_t* d_inst_base = nullptr;      // [n_inst+1]
  int* d_ilist = nullptr;              // [2][n_pad]
  int* d_icnt = nullptr;               // [2][n_inst]
  int* d_bt0 = nullptr;                // [n_blocks+1]
  int* d_binst = nullptr;              // [n_blocks]
  int* d_blb = nullptr;                // [n_blocks]
  int* d_ifb = nullptr;                // [n_inst] first block of each instance
  int64_t* d_boff = nullptr;           // [n_pad+1]
  int32_t* d_blk2 = nullptr;
  int own_blocks = 0, own_bmax = 0, own_targets = 0, own_inst_max = 0;
  // input record of an adjoint's forward (owned by that mc_adjoint call)
  long long* d_xrec = nullptr;
  long long xrec_step0 = 0, xrec_steps = 0;
  // checkpoints of an adjoint's forward, stored by the update kernels
  double* d_ck_y = nullptr;
  double* d_ck_I = nullptr;
  int32_t* d_ck_r = nullptr;
  long long ck_step0 = 0, ck_every = 1, ck_count = 0;
  unsigned long long* d_phase = nullptr;
  bool phase_on = false;
  std::vector<double> phase_wg;        // per-workgroup phase times (us/step) of the last mc_profile_phases
  unsigned* d_nb = nullptr;            // near table offsets [n_pad][pG+1]
  unsigned long long* d_ne = nullptr;  // near table entries
  // recording
  int n_wg = 0;
  int qpw = 0;
  int wg_neurons = 0;                  // neurons updated by one workgroup (raster bound)
  int2* d_raster = nullptr;
  long long raster_cap = 0;            // per workgroup
  long long* d_raster_cnt = nullptr;
  unsigned long long* d_wg_events = nullptr;
  unsigned long long* d_wg_spikes = nullptr;
  unsigned* d_overflow = nullptr;
  unsigned* d_wbad = nullptr;          // weight update check flag
  int64_t cap_steps = 0;               // steps the raster segments can absorb between drains
  int64_t steps_since_drain = 0;
  // drained raster (dense ids), sorted by (step, id); a deque, so that growing
  // it never copies the spikes already held (long runs hold tens of millions)
  std::deque<int32_t> r_step, r_id;
  int64_t events_base = 0;
  std::vector<int64_t> spikes_base;
  int64_t step = 0;
  mc_launch launch{};
  // graph
  hipGraphExec_t graph = nullptr;
  int graph_steps = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_mid = nullptr;
  // HIP events around every persistent-kernel launch of the latest
  // mc_simulate (pairs k, k+1; at most kLaunchEvents / 2 launches timed);
  // a call that is one launch is timed by ev0 and ev1 (whole_call)
  std::vector<hipEvent_t> ev_launch;
  bool whole_call = false;
  std::vector<unsigned char> dq;       // 1024 quantiles of the store's delay histogram (atomic probe)
  int launches_timed = 0;
  int64_t steps_timed = 0;
  hipStream_t aux = nullptr;           // read-back of the raster beside the simulation stream
  int2* d_pack = nullptr;              // raster prefixes packed for one read-back
  int64_t pack_cap = 0;
  long long* d_pack_off = nullptr;     // [n_wg+1]
  int64_t pack_off_cap = 0;
  void* h_stage = nullptr;             // pinned staging of the adjoint's work lists
  size_t stage_bytes = 0;
  double last_ms = 0.0;
  double adj_forward_ms = 0.0, adj_reverse_ms = 0.0;

  DevNet dev() const {
    DevNet p{};
    p.n_pad = n_pad; p.n_quads = n_quads; p.ring_stride = ring_stride; p.n_pops = h.n_pops;
    p.row_ptr = d_row_ptr; p.tgt = d_tgt; p.wq = d_wq; p.dly = d_dly;
    p.y = d_y; p.I = d_I; p.r = d_r; p.ring = d_ring;
    p.qseed = d_qseed; p.qlocal = d_qlocal; p.qpops = d_qpops; p.table = d_table;
    p.P11 = h.P11; p.P21 = h.P21; p.P22 = h.P22; p.P20 = h.P20; p.i_e = h.i_e; p.theta = h.theta; p.y_reset = h.y_reset;
    p.jext_q = h.jext_q; p.ref_steps = h.ref_steps;
    p.step_base = d_step;
    p.raster = d_raster; p.raster_cap = raster_cap; p.raster_cnt = d_raster_cnt;
    p.wg_events = d_wg_events; p.wg_spikes = d_wg_spikes; p.overflow = d_overflow;
    p.n_inst = h.n_inst; p.qinst = d_qinst; p.inst_base = d_inst_base; p.ilist = d_ilist; p.icnt = d_icnt;
    p.xrec = d_xrec; p.xrec_step0 = xrec_step0; p.xrec_steps = xrec_steps;
    p.ck_y = d_ck_y; p.ck_I = d_ck_I; p.ck_r = d_ck_r;
    p.ck_step0 = ck_step0; p.ck_every = ck_every; p.ck_count = ck_count;
    return p;
  }

  BucketArgs bucket() const {
    BucketArgs a{};
    a.G = own_blocks; a.B = wg_neurons;
    a.bt0 = d_bt0; a.binst = d_binst; a.blb = d_blb; a.ifb = d_ifb; a.boff = d_boff; a.blk2 = d_blk2;
    a.flags = d_flags; a.pub = d_pub; a.bk = d_bk; a.cap = bk_cap;
    a.wait_ticks = (long long)wall_khz * 1000 * kWaitSeconds;
    a.horizon = horizon;
    a.phase = phase_on ? d_phase : nullptr;
    a.inst_wg_max = own_inst_max;
    return a;
  }

  OwnerArgs owner() const {
    OwnerArgs a{};
    a.n_blocks = own_blocks; a.bmax = own_bmax;
    a.bt0 = d_bt0; a.binst = d_binst; a.blb = d_blb; a.boff = d_boff; a.blk2 = d_blk2;
    return a;
  }

  PersistArgs persist() const {
    PersistArgs a{};
    a.G = pG; a.B = pB; a.DL = pDL; a.BW = (pB + 31) / 32;
    a.horizon = horizon;
    a.bstart = d_bstart;
    a.blk = d_blk; a.flags = d_flags; a.pub = d_pub;
    a.wait_ticks = (long long)wall_khz * 1000 * kWaitSeconds;
    a.phase = phase_on ? d_phase : nullptr;
    a.nb = d_nb; a.ne = d_ne;
    if (const char* lc = getenv("MC_PERSIST_LIST_CAP")) a.list_cap = std::max(0, atoi(lc));
    return a;
  }

  // dense id -> instance
  int inst_of(int64_t dense) const {
    return (int)(std::upper_bound(h.inst_off.begin(), h.inst_off.end(), dense) - h.inst_off.begin()) - 1;
  }
  int64_t pad_of(int64_t dense) const {
    const int b = inst_of(dense);
    return dense - h.inst_off[b] + inst_off_pad[b];
  }
  int64_t dense_of(int64_t padded) const {
    const int b = (int)(std::upper_bound(inst_off_pad.begin(), inst_off_pad.end(), padded) - inst_off_pad.begin()) - 1;
    const int64_t local = padded - inst_off_pad[b];
    if (local >= h.inst_off[b + 1] - h.inst_off[b]) return -1;
    return h.inst_off[b] + local;
  }
};

namespace {

bool usable(mc_net* n) { return n && !n->failed; }
bool device_ready(mc_net* n) { return usable(n) && !n->host_only; }

int release_recording(mc_net* n) {
  dev_free(n->alloc, n->d_raster);
  dev_free(n->alloc, n->d_raster_cnt);
  dev_free(n->alloc, n->d_wg_events);
  dev_free(n->alloc, n->d_wg_spikes);
  return MC_OK;
}

void release_all(mc_net* n) {
  if (n->graph) { (void)hipGraphExecDestroy(n->graph); n->graph = nullptr; }
  release_recording(n);
  dev_free(n->alloc, n->d_blk); dev_free(n->alloc, n->d_flags); dev_free(n->alloc, n->d_pub); dev_free(n->alloc, n->d_phase);
  dev_free(n->alloc, n->d_nb); dev_free(n->alloc, n->d_bk);
  dev_free(n->alloc, n->d_ne);
  dev_free(n->alloc, n->d_bstart);
  dev_free(n->alloc, n->d_qinst); dev_free(n->alloc, n->d_inst_base); dev_free(n->alloc, n->d_ilist); dev_free(n->alloc, n->d_icnt);
  dev_free(n->alloc, n->d_bt0); dev_free(n->alloc, n->d_binst); dev_free(n->alloc, n->d_blb); dev_free(n->alloc, n->d_ifb); dev_free(n->alloc, n->d_boff);
  dev_free(n->alloc, n->d_blk2);
  dev_free(n->alloc, n->d_overflow);
  dev_free(n->alloc, n->d_wbad);
  dev_free(n->alloc, n->d_row_ptr); dev_free(n->alloc, n->d_tgt); dev_free(n->alloc, n->d_wq); dev_free(n->alloc, n->d_dly);
  dev_free(n->alloc, n->d_y); dev_free(n->alloc, n->d_I); dev_free(n->alloc, n->d_r); dev_free(n->alloc, n->d_ring);
  dev_free(n->alloc, n->d_qseed); dev_free(n->alloc, n->d_qlocal); dev_free(n->alloc, n->d_qpops); dev_free(n->alloc, n->d_table); dev_free(n->alloc, n->d_step);
  if (n->ev0) { (void)hipEventDestroy(n->ev0); n->ev0 = nullptr; }
  if (n->ev1) { (void)hipEventDestroy(n->ev1); n->ev1 = nullptr; }
  if (n->ev_mid) { (void)hipEventDestroy(n->ev_mid); n->ev_mid = nullptr; }
  for (hipEvent_t e : n->ev_launch) (void)hipEventDestroy(e);
  n->ev_launch.clear();
  dev_free(n->alloc, n->d_pack); dev_free(n->alloc, n->d_pack_off);
  n->pack_cap = 0; n->pack_off_cap = 0;
  if (n->h_stage) { (void)hipHostFree(n->h_stage); n->h_stage = nullptr; n->stage_bytes = 0; }
  if (n->aux) { (void)hipStreamDestroy(n->aux); n->aux = nullptr; }
  if (n->own_stream && n->stream) { (void)hipStreamDestroy(n->stream); n->stream = nullptr; }
}

// Spikes a workgroup of `neurons` can emit in `steps` steps: each neuron at
// most once per (t_ref/h + 1) steps.
int64_t spike_bound(int64_t neurons, int64_t steps, int ref) {
  return neurons * ((steps + ref) / (ref + 1));
}

// Copies the private raster segments to the host list (sorted by step, id)
// and empties them.  Waits for `upto` (an event on the simulation stream) if
// given, else for the whole simulation stream; the read-back itself runs on
// the second stream, so work queued after `upto` keeps running.
int drain(mc_net* n, hipEvent_t upto = nullptr) {
  if (!n->d_raster) return MC_OK;
  if (upto) HIP_TRY(hipEventSynchronize(upto));
  else HIP_TRY(hipStreamSynchronize(n->stream));
  hipStream_t s = n->aux;
  unsigned ovf = 0;
  std::vector<long long> cnt((size_t)n->n_wg);
  HIP_TRY(hipMemcpyAsync(&ovf, n->d_overflow, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(cnt.data(), n->d_raster_cnt, sizeof(long long) * n->n_wg, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (ovf & kErrWaitTimeout) {
    n->failed = true;
    return set_error(MC_ERR_TIMEOUT, "persistent kernel: a workgroup waited more than " + std::to_string(kWaitSeconds) +
                                         " s for the spike records of a step and the launch was abandoned");
  }
  if (ovf & kErrRasterOverflow) {
    n->failed = true;
    return set_error(MC_ERR_STATE, "raster segment overflow (internal capacity error)");
  }
  std::vector<long long> seg_off((size_t)n->n_wg + 1, 0);
  for (int g = 0; g < n->n_wg; ++g) seg_off[g + 1] = seg_off[g] + cnt[g];
  const long long total = seg_off[n->n_wg];
  std::vector<int2> buf((size_t)total);
  if (total > 0) {
    // the used prefixes packed on the device, then one copy
    int rc;
    if (n->pack_off_cap < n->n_wg + 1) {
      dev_free(n->alloc, n->d_pack_off);
      n->pack_off_cap = 0;
      if ((rc = dev_alloc(n->alloc, &n->d_pack_off, (size_t)n->n_wg + 1)) != MC_OK) return rc;
      n->pack_off_cap = n->n_wg + 1;
    }
    if (n->pack_cap < total) {
      dev_free(n->alloc, n->d_pack);
      n->pack_cap = 0;
      if ((rc = dev_alloc(n->alloc, &n->d_pack, (size_t)total)) != MC_OK) return rc;
      n->pack_cap = total;
    }
    HIP_TRY(hipMemcpyAsync(n->d_pack_off, seg_off.data(), sizeof(long long) * (n->n_wg + 1), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_raster_pack(n->d_raster, n->raster_cap, n->d_pack_off, n->n_wg, n->d_pack, s));
    HIP_TRY(hipMemcpyAsync(buf.data(), n->d_pack, sizeof(int2) * total, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipMemsetAsync(n->d_raster_cnt, 0, sizeof(long long) * n->n_wg, s));
  HIP_TRY(hipStreamSynchronize(s));
  // Workgroup g's segment holds its own neurons, whose ids all exceed those
  // of workgroups < g, by step; a stable counting sort by step over the
  // segments in order groups a step's spikes by workgroup.  The persistent
  // and step kernels write a step's ids in ascending order, the bucket
  // kernel in any order: a step whose ids are not ascending is sorted.
  if (total > 0) {
    int smin = buf[0].x, smax = buf[0].x;
    for (const int2& e : buf) { smin = std::min(smin, e.x); smax = std::max(smax, e.x); }
    std::vector<size_t> pos((size_t)(smax - smin) + 2, 0);
    for (const int2& e : buf) ++pos[(size_t)(e.x - smin) + 1];
    for (size_t k = 1; k < pos.size(); ++k) pos[k] += pos[k - 1];
    const std::vector<size_t> first(pos);
    const size_t base = n->r_step.size();
    n->r_step.resize(base + (size_t)total);
    n->r_id.resize(base + (size_t)total);
    for (const int2& e : buf) {
      const size_t k = base + pos[(size_t)(e.x - smin)]++;
      n->r_step[k] = e.x;
      n->r_id[k] = (int32_t)n->dense_of(e.y);
    }
    for (size_t k = 0; k + 1 < first.size(); ++k) {
      auto b = n->r_id.begin() + (std::ptrdiff_t)(base + first[k]), e = n->r_id.begin() + (std::ptrdiff_t)(base + first[k + 1]);
      if (!std::is_sorted(b, e)) std::sort(b, e);
    }
  }
  n->steps_since_drain = 0;
  return MC_OK;
}

// Folds the per-workgroup counters into the host base (before they are
// reallocated for a new launch shape).
int fold_counters(mc_net* n) {
  if (!n->d_wg_events) return MC_OK;
  HIP_TRY(hipStreamSynchronize(n->stream));
  std::vector<unsigned long long> ev((size_t)n->n_wg), sp((size_t)n->n_wg * n->h.n_pops);
  HIP_TRY(hipMemcpy(ev.data(), n->d_wg_events, sizeof(unsigned long long) * ev.size(), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(sp.data(), n->d_wg_spikes, sizeof(unsigned long long) * sp.size(), hipMemcpyDeviceToHost));
  for (auto v : ev) n->events_base += (int64_t)v;
  for (int g = 0; g < n->n_wg; ++g)
    for (int a = 0; a < n->h.n_pops; ++a) n->spikes_base[a] += (int64_t)sp[(size_t)g * n->h.n_pops + a];
  HIP_TRY(hipMemsetAsync(n->d_wg_events, 0, sizeof(unsigned long long) * ev.size(), n->stream));
  HIP_TRY(hipMemsetAsync(n->d_wg_spikes, 0, sizeof(unsigned long long) * sp.size(), n->stream));
  return MC_OK;
}

// (Re)allocates the recording buffers for the current launch shape with room
// for `steps` steps between drains.
int setup_recording(mc_net* n, int64_t steps) {
  int rc;
  if ((rc = drain(n)) != MC_OK) return rc;
  if ((rc = fold_counters(n)) != MC_OK) return rc;
  // a captured graph holds the old buffer addresses
  if (n->graph) { (void)hipGraphExecDestroy(n->graph); n->graph = nullptr; }
  const int64_t old_steps = n->cap_steps;
  release_recording(n);
  auto alloc = [&](int64_t s) {
    n->raster_cap = spike_bound(n->wg_neurons, s, n->h.ref_steps) + 1;
    n->cap_steps = s;
    int r = dev_alloc(n->alloc, &n->d_raster, (size_t)n->n_wg * n->raster_cap);
    if (r == MC_OK) r = dev_alloc(n->alloc, &n->d_raster_cnt, (size_t)n->n_wg);
    if (r == MC_OK) r = dev_alloc(n->alloc, &n->d_wg_events, (size_t)n->n_wg);
    if (r == MC_OK) r = dev_alloc(n->alloc, &n->d_wg_spikes, (size_t)n->n_wg * n->h.n_pops);
    if (r != MC_OK) { release_recording(n); n->cap_steps = 0; n->raster_cap = 0; }
    return r;
  };
  if ((rc = alloc(steps)) != MC_OK) {
    // keep the handle usable with the capacity it had, if there was one
    const std::string msg = g_last_error;
    if (old_steps > 0 && old_steps < steps && alloc(old_steps) == MC_OK) {
      rc = set_error(rc, msg + " (recording capacity left at " + std::to_string(old_steps) + " steps)");
    } else {
      n->failed = true;
      return rc;
    }
  }
  HIP_TRY(hipMemsetAsync(n->d_raster_cnt, 0, sizeof(long long) * n->n_wg, n->stream));
  HIP_TRY(hipMemsetAsync(n->d_wg_events, 0, sizeof(unsigned long long) * n->n_wg, n->stream));
  HIP_TRY(hipMemsetAsync(n->d_wg_spikes, 0, sizeof(unsigned long long) * n->n_wg * n->h.n_pops, n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  n->steps_since_drain = 0;
  return rc;
}

int validate_launch(const mc_net* n, const mc_launch& l) {
  if (l.struct_size != sizeof(mc_launch)) return set_error(MC_ERR_INVALID_ARG, "mc_launch.struct_size mismatch");
  if (l.scheme != MC_SCHEME_STEP_KERNELS && l.scheme != MC_SCHEME_PERSISTENT_LDS && l.scheme != MC_SCHEME_TARGET_OWNER &&
      l.scheme != MC_SCHEME_PERSISTENT_BUCKETS)
    return set_error(MC_ERR_INVALID_ARG, "unknown scheme");
  if (l.scheme == MC_SCHEME_PERSISTENT_BUCKETS) {
    if (l.block < 64 || l.block > kBucketMaxBlock || l.block % 64)
      return set_error(MC_ERR_INVALID_ARG, "the bucket scheme runs 64..512 threads per workgroup");
    if (l.neurons_per_wg < 0 || l.neurons_per_wg % 4 || l.neurons_per_wg > std::min(kBucketMaxB, 64 * l.block))
      return set_error(MC_ERR_INVALID_ARG, "bucket scheme: neurons_per_wg must be a multiple of 4, <= min(4092, 64 x block)");
    if (l.steps_per_graph < 0 || l.steps_per_graph > 100000) return set_error(MC_ERR_INVALID_ARG, "steps_per_graph out of [0, 100000]");
    if (l.rows_per_wave != 0 && l.rows_per_wave != 1) return set_error(MC_ERR_INVALID_ARG, "rows_per_wave must be 0 or 1");
    return MC_OK;
  }
  if (l.block < 64 || l.block > 1024 || l.block % 64) return set_error(MC_ERR_INVALID_ARG, "block must be a multiple of 64 in [64, 1024]");
  if (l.scheme == MC_SCHEME_PERSISTENT_LDS && l.block > kPersistMaxBlock)
    return set_error(MC_ERR_INVALID_ARG, "the persistent scheme runs at most 512 threads per workgroup");
  const int npw = l.neurons_per_wg;
  const int npw_max = l.scheme == MC_SCHEME_PERSISTENT_LDS ? std::min(l.block, kPersistMaxB)
                                                           : std::min(4 * l.block, 4 * kMaxQuadsPerWgHost);
  if (npw < 0 || npw % 4 || npw > npw_max)
    return set_error(MC_ERR_INVALID_ARG, "neurons_per_wg must be a multiple of 4, <= min(4*block, 1024) (step "
                                         "kernels) or <= block (persistent)");
  if (l.steps_per_graph < 0 || l.steps_per_graph > 100000) return set_error(MC_ERR_INVALID_ARG, "steps_per_graph out of [0, 100000]");
  if (l.rows_per_wave != 0 && l.rows_per_wave != 1) return set_error(MC_ERR_INVALID_ARG, "rows_per_wave must be 0 or 1");
  (void)n;
  return MC_OK;
}

// Shape of the persistent scheme: G co-resident workgroups, workgroup g owning
// targets [bs[g], bs[g+1]) (B of them, the last block possibly fewer), DL
// near steps of input in LDS (as many as the LDS holds, <= 101).
// neurons_per_wg = 0: one workgroup per compute unit.  (Blocks sized to
// equalise the expected synaptic input per workgroup were measured slower on
// the full microcircuit: the larger blocks leave fewer delay steps in LDS.)
int persist_shape(mc_net* n, const mc_launch& l, int* G, int* B, int* DL, std::vector<int>& bs) {
  const int64_t P = n->n_pad;
  const int cap = std::min(kPersistMaxB, l.block);
  int b = l.neurons_per_wg;
  if (b == 0) {
    const int g0 = (int)std::max<int64_t>(1, std::min<int64_t>(std::min(n->n_cu, l.block), P / 4));
    b = (int)align_up((P + g0 - 1) / g0, 4);
  }
  if (b > cap) return set_error(MC_ERR_RANGE, "network too large for the persistent LDS scheme at this block size");
  const int g = (int)((P + b - 1) / b);
  bs.assign((size_t)g + 1, 0);
  for (int k = 0; k <= g; ++k) bs[k] = (int)std::min<int64_t>((int64_t)k * b, P);
  if (g > 2 * l.block || g > kPersistMaxBlock)
    return set_error(MC_ERR_RANGE, "persistent scheme needs workgroups <= 2 x threads per workgroup and <= 512");
  size_t stat = 0;
  HIP_TRY(persist_static_lds(&stat));
  const size_t base = persist_lds_bytes(g, b, 0);
  // workgroups that must share a compute unit divide its LDS
  const int per_cu = (g + n->n_cu - 1) / n->n_cu;
  const size_t budget = (size_t)n->lds_max / per_cu;
  if (stat + base + 2 * (size_t)b * 8 > budget) return set_error(MC_ERR_RANGE, "LDS too small for the persistent scheme");
  const int dl = (int)std::min<size_t>(101, (budget - stat - base) / ((size_t)b * 8));
  const size_t lds = persist_lds_bytes(g, b, dl);
  HIP_TRY(persist_set_lds_limit(lds));
  int occ = 0;
  HIP_TRY(persist_occupancy(l.block, lds, &occ));
  if (occ < 1 || g > n->n_cu * occ)
    return set_error(MC_ERR_RANGE, "persistent workgroups would not all be co-resident");
  *G = g; *B = b; *DL = dl;
  return MC_OK;
}

// Blocks of at most `targets` targets (a multiple of 4) that every
// instance's padded range is split into (no block spans two instances).
int64_t owner_block_count(const mc_net* n, int targets) {
  if (targets <= 0) return 0;
  int64_t G = 0;
  for (int b = 0; b < n->h.n_inst; ++b)
    G += std::max<int64_t>(1, (n->inst_off_pad[b + 1] - n->inst_off_pad[b] + targets - 1) / targets);
  return G;
}

// Targets per workgroup of the bucket scheme: neurons_per_wg, or (0) the
// smallest multiple of 4 for which all workgroups are co-resident.  Every
// instance may have at most kBucketMaxProducers workgroups and at most two
// per thread (the listing of a step with more spikes than the LDS list
// holds sums two producers per thread).
int bucket_shape(mc_net* n, const mc_launch& l, int* B_out) {
  const int bmax = std::min(kBucketMaxB, 64 * l.block);   // at most 16 quads per thread
  if (bucket_lds_bytes(bmax) > (size_t)n->lds_max && bucket_lds_bytes(4) > (size_t)n->lds_max)
    return set_error(MC_ERR_RANGE, "bucket scheme: LDS too small");
  HIP_TRY(bucket_set_lds_limit(std::min<size_t>((size_t)n->lds_max, bucket_lds_bytes(bmax))));
  auto fits = [&](int B, std::string* why) -> bool {
    int occ = 0;
    const int64_t G = owner_block_count(n, B);
    int64_t gmax = 0;
    for (int b = 0; b < n->h.n_inst; ++b)
      gmax = std::max<int64_t>(gmax, (n->inst_off_pad[b + 1] - n->inst_off_pad[b] + B - 1) / B);
    if (bucket_lds_bytes(B) <= (size_t)n->lds_max &&
        bucket_occupancy(B, l.block, (int)std::min<int64_t>(gmax, kBucketMaxProducers), &occ) != hipSuccess) {
      (void)hipGetLastError();
      occ = 0;
    }
    if (gmax > kBucketMaxProducers || gmax > 2 * l.block) {
      if (why) *why = "an instance would have more than min(512, 2 x threads) workgroups";
      return false;
    }
    if (occ < 1 || G > (int64_t)n->n_cu * occ) {
      if (why) *why = "bucket workgroups would not all be co-resident";
      return false;
    }
    return true;
  };
  std::string why;
  if (l.neurons_per_wg) {
    if (l.neurons_per_wg > bmax) return set_error(MC_ERR_RANGE, "bucket scheme: at most min(4092, 64 x threads) targets per workgroup");
    if (!fits(l.neurons_per_wg, &why)) return set_error(MC_ERR_RANGE, "bucket scheme: " + why);
    *B_out = l.neurons_per_wg;
    return MC_OK;
  }
  // the smallest block for which every workgroup is co-resident: several
  // per compute unit where registers and LDS allow (the search starts at
  // sixteen per compute unit)
  int B = (int)align_up(std::max<int64_t>(4, (n->n_pad + (int64_t)n->n_cu * 16 - 1) / ((int64_t)n->n_cu * 16)), 4);
  for (; B <= bmax; B += 4)
    if (fits(B, &why)) { *B_out = B; return MC_OK; }
  return set_error(MC_ERR_RANGE, "bucket scheme: no co-resident shape for this network at this block size");
}

// Target blocks of the owner kernel and of the bucket kernel: every
// instance's padded range split into owner_block_count blocks of whole quads
// of at most `targets` targets, and each row's sub-row bounds for the blocks
// of its own instance.
int setup_owner(mc_net* n, int targets, int max_targets) {
  if (targets < 4 || targets % 4) return set_error(MC_ERR_INVALID_ARG, "target blocks need a positive multiple of 4 targets");
  const int ni = n->h.n_inst;
  std::vector<int> bt0, binst, blb, ifb((size_t)ni);
  for (int b = 0; b < ni; ++b) {
    const int64_t p0 = n->inst_off_pad[b], L = n->inst_off_pad[b + 1] - p0;
    const int64_t G = std::max<int64_t>(1, (L + targets - 1) / targets);
    ifb[b] = (int)bt0.size();
    for (int64_t j = 0; j < G; ++j) {
      bt0.push_back((int)(p0 + 4 * ((L / 4) * j / G)));
      binst.push_back(b);
      blb.push_back((int)j);
    }
  }
  const int nb = (int)bt0.size();
  bt0.push_back((int)n->n_pad);
  int bmax = 1;
  for (int k = 0; k < nb; ++k) bmax = std::max(bmax, bt0[k + 1] - bt0[k]);
  if (bmax > max_targets) return set_error(MC_ERR_INVALID_ARG, "target blocks hold at most " + std::to_string(max_targets) + " targets");
  std::vector<int64_t> boff((size_t)n->n_pad + 1, 0);
  int inst_max = 1;
  for (int b = 0; b < ni; ++b) {
    const int nblk = ((b + 1 < ni) ? ifb[b + 1] : nb) - ifb[b];
    inst_max = std::max(inst_max, nblk);
    for (int64_t i = n->inst_off_pad[b]; i < n->inst_off_pad[b + 1]; ++i) boff[i + 1] = boff[i] + nblk + 1;
  }
  int rc;
  dev_free(n->alloc, n->d_bt0); dev_free(n->alloc, n->d_binst); dev_free(n->alloc, n->d_blb); dev_free(n->alloc, n->d_ifb); dev_free(n->alloc, n->d_boff);
  dev_free(n->alloc, n->d_blk2);
  if ((rc = dev_alloc(n->alloc, &n->d_bt0, (size_t)nb + 1)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_binst, (size_t)nb)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_blb, (size_t)nb)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_ifb, (size_t)ni)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_boff, (size_t)n->n_pad + 1)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_blk2, (size_t)boff[n->n_pad])) != MC_OK) return rc;
  HIP_TRY(hipMemcpy(n->d_bt0, bt0.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_binst, binst.data(), sizeof(int) * nb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_blb, blb.data(), sizeof(int) * nb, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_ifb, ifb.data(), sizeof(int) * ni, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_boff, boff.data(), sizeof(int64_t) * (n->n_pad + 1), hipMemcpyHostToDevice));
  HIP_TRY(launch_build_blk2(n->d_row_ptr, n->d_tgt, n->n_pad, n->d_boff, n->d_qinst, n->d_ifb, n->d_bt0, n->d_blk2,
                            n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  n->own_blocks = nb;
  n->own_bmax = bmax;
  n->own_inst_max = inst_max;
  n->own_targets = targets;
  return MC_OK;
}

int apply_launch(mc_net* n, const mc_launch& l) {
  int rc = validate_launch(n, l);
  if (rc != MC_OK) return rc;
  int qpw = 0, n_wg = 0, wg_neurons = 0, G = 0, B = 0, DL = 0;
  std::vector<int> bs;
  if (l.scheme == MC_SCHEME_STEP_KERNELS || l.scheme == MC_SCHEME_TARGET_OWNER) {
    // step kernels: neurons_per_wg / 4 quads per workgroup; target owner: one
    // quad per thread in the update kernel, neurons_per_wg sizes the delivery blocks
    qpw = l.scheme == MC_SCHEME_TARGET_OWNER ? std::min(l.block, kMaxQuadsPerWgHost) : l.neurons_per_wg / 4;
    if (qpw == 0) qpw = std::min<int>(l.block, 64);
    n_wg = (int)((n->n_quads + qpw - 1) / qpw);
    wg_neurons = 4 * qpw;
  } else if (l.scheme == MC_SCHEME_PERSISTENT_LDS) {
    if ((rc = persist_shape(n, l, &G, &B, &DL, bs)) != MC_OK) return rc;
    n_wg = G;
    wg_neurons = B;
  } else {
    if ((rc = bucket_shape(n, l, &B)) != MC_OK) return rc;
    G = (int)owner_block_count(n, B);
    n_wg = G;
    wg_neurons = B;
  }
  const bool shape_changed = (l.scheme != n->launch.scheme || n_wg != n->n_wg || wg_neurons != n->wg_neurons ||
                              (l.scheme == MC_SCHEME_PERSISTENT_LDS && bs != n->bstart_host) ||
                              (l.scheme == MC_SCHEME_TARGET_OWNER &&
                               n->own_targets != (l.neurons_per_wg ? l.neurons_per_wg : 256)) ||
                              (l.scheme == MC_SCHEME_PERSISTENT_BUCKETS && n->own_targets != B));
  if (n->graph && (shape_changed || l.steps_per_graph != n->graph_steps || l.block != n->launch.block ||
                   l.rows_per_wave != n->launch.rows_per_wave)) {
    (void)hipGraphExecDestroy(n->graph);
    n->graph = nullptr;
  }
  if (shape_changed || !n->d_raster) {
    // the old shape's buffers go first: a failure from here on leaves no
    // consistent shape, so it marks the handle failed
    struct FailGuard {
      mc_net* n; bool armed = true;
      ~FailGuard() { if (armed) n->failed = true; }
    } guard{n};
    if ((rc = drain(n)) != MC_OK) return rc;
    if ((rc = fold_counters(n)) != MC_OK) return rc;
    release_recording(n);   // sized for the old shape
    if (l.scheme == MC_SCHEME_PERSISTENT_LDS) {
      dev_free(n->alloc, n->d_blk); dev_free(n->alloc, n->d_flags); dev_free(n->alloc, n->d_pub); dev_free(n->alloc, n->d_bstart);
      if ((rc = dev_alloc(n->alloc, &n->d_blk, (size_t)n->n_pad * (G + 1))) != MC_OK) return rc;
      if ((rc = dev_alloc(n->alloc, &n->d_flags, persist_flag_words(G))) != MC_OK) return rc;
      if ((rc = dev_alloc(n->alloc, &n->d_pub, (size_t)G * kRecSlots * B)) != MC_OK) return rc;
      if ((rc = dev_alloc(n->alloc, &n->d_bstart, (size_t)G + 1)) != MC_OK) return rc;
      HIP_TRY(hipMemcpy(n->d_bstart, bs.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice));
      n->bstart_host = bs;
      HIP_TRY(launch_build_blk(n->d_row_ptr, n->d_tgt, n->n_pad, G, n->d_bstart, n->d_blk, n->stream));
      HIP_TRY(hipMemsetAsync(n->d_flags, 0, sizeof(unsigned long long) * persist_flag_words(G), n->stream));
      // near table: the delay-1/2 synapses per (source, workgroup), CSR
      dev_free(n->alloc, n->d_nb); dev_free(n->alloc, n->d_ne);
      const size_t cells = (size_t)n->n_pad * (G + 1);
      if ((rc = dev_alloc(n->alloc, &n->d_nb, cells)) != MC_OK) return rc;
      HIP_TRY(launch_near_count(n->d_tgt, n->d_dly, n->d_blk, n->n_pad, G, n->d_nb, n->stream));
      std::vector<unsigned> hc;
      try { hc.resize(cells); } catch (...) { return set_error(MC_ERR_OOM, "host allocation of the near-table offsets failed"); }
      HIP_TRY(hipStreamSynchronize(n->stream));
      HIP_TRY(hipMemcpy(hc.data(), n->d_nb, sizeof(unsigned) * cells, hipMemcpyDeviceToHost));
      uint64_t total = 0;
      for (size_t k = 0; k < cells; ++k) { const unsigned c = hc[k]; hc[k] = (unsigned)total; total += c; }
      if (total >= ((uint64_t)1 << 32)) return set_error(MC_ERR_RANGE, "more than 2^32 delay-1/2 synapses");
      HIP_TRY(hipMemcpy(n->d_nb, hc.data(), sizeof(unsigned) * cells, hipMemcpyHostToDevice));
      if ((rc = dev_alloc(n->alloc, &n->d_ne, (size_t)std::max<uint64_t>(total, 1))) != MC_OK) return rc;
      HIP_TRY(launch_near_fill(n->d_tgt, n->d_wq, n->d_dly, n->d_blk, n->d_bstart, n->n_pad, G, n->d_nb, n->d_ne,
                               n->stream));
      HIP_TRY(hipStreamSynchronize(n->stream));
    }
    if (l.scheme == MC_SCHEME_TARGET_OWNER &&
        (rc = setup_owner(n, l.neurons_per_wg ? l.neurons_per_wg : 256, kOwnerMaxTargets)) != MC_OK)
      return rc;
    if (l.scheme == MC_SCHEME_PERSISTENT_BUCKETS) {
      if ((rc = setup_owner(n, B, kBucketMaxB)) != MC_OK) return rc;
      G = n->own_blocks;
      dev_free(n->alloc, n->d_flags); dev_free(n->alloc, n->d_pub); dev_free(n->alloc, n->d_bk);
      n->bk_cap = kBucketCap;
      if ((rc = dev_alloc(n->alloc, &n->d_flags, persist_flag_words(G))) != MC_OK) return rc;
      if ((rc = dev_alloc(n->alloc, &n->d_pub, (size_t)G * kRecSlots * B)) != MC_OK) return rc;
      if ((rc = dev_alloc(n->alloc, &n->d_bk, (size_t)G * kRingSlots * n->bk_cap)) != MC_OK) return rc;
      HIP_TRY(hipMemsetAsync(n->d_flags, 0, sizeof(unsigned long long) * persist_flag_words(G), n->stream));
      HIP_TRY(hipStreamSynchronize(n->stream));
    }
    n->qpw = qpw;
    n->n_wg = n_wg;
    n->wg_neurons = wg_neurons;
    // the LDS-window scheme's shape (its tables are rebuilt whenever it is set again)
    const bool lds_scheme = l.scheme == MC_SCHEME_PERSISTENT_LDS;
    n->pG = lds_scheme ? G : 0; n->pB = lds_scheme ? B : 0; n->pDL = lds_scheme ? DL : 0;
    n->launch = l;
    guard.armed = false;   // setup_recording keeps the handle usable on its own failures where it can
    if ((rc = setup_recording(n, std::max<int64_t>(n->cap_steps, 4096))) != MC_OK) return rc;
  }
  n->launch = l;
  return MC_OK;
}

// Enqueues `count` steps directly (no graph) on stream s.
hipError_t enqueue_direct(mc_net* n, int count, hipStream_t s) {
  const DevNet p = n->dev();
  hipError_t e = hipSuccess;
  if (n->launch.scheme == MC_SCHEME_STEP_KERNELS) {
    for (int k = 0; k < count && e == hipSuccess; ++k)
      e = launch_step(p, k, n->qpw, n->n_wg, n->launch.block, n->launch.rows_per_wave, s);
  } else if (n->launch.scheme == MC_SCHEME_TARGET_OWNER) {
    const OwnerArgs a = n->owner();
    e = launch_zero_lists(n->d_icnt, 2 * n->h.n_inst, s);
    for (int k = 0; k < count && e == hipSuccess; ++k) {
      e = launch_step_lists(p, k, n->qpw, n->n_wg, n->launch.block, s);
      if (e == hipSuccess) e = launch_owner(p, a, k, s);
    }
  } else if (n->launch.scheme == MC_SCHEME_PERSISTENT_BUCKETS) {
    return launch_bucket(p, n->bucket(), count, n->launch.block, s);     // advances the step counter itself
  } else {
    return launch_persist(p, n->persist(), count, n->launch.block, s);   // advances the step counter itself
  }
  if (e == hipSuccess) e = launch_advance(n->d_step, count, s);
  return e;
}

int build_graph(mc_net* n) {
  if (n->graph) return MC_OK;
  hipStream_t cs;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const int S = n->launch.steps_per_graph;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    e = enqueue_direct(n, S, cs);
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&n->graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) { n->graph = nullptr; return set_error(MC_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e)); }
  n->graph_steps = S;
  return MC_OK;
}

constexpr int kLaunchEvents = 128;

// Records the event that opens (begin) or closes a timed persistent launch on
// the simulation stream; beyond kLaunchEvents / 2 launches nothing is timed.
// A launch that is a whole mc_simulate call (`whole`: nothing else between the
// call's events ev0 and ev1) records nothing and is timed by those two: every
// event on the stream lengthens the call by ~4.5 us, a few per cent of a
// 20-step call.
int launch_event(mc_net* n, bool begin, int64_t steps, bool whole = false) {
  if ((n->launch.scheme != MC_SCHEME_PERSISTENT_LDS && n->launch.scheme != MC_SCHEME_PERSISTENT_BUCKETS) ||
      n->ev_launch.size() < (size_t)kLaunchEvents)
    return MC_OK;
  if (whole) {
    if (!begin) { n->whole_call = true; n->launches_timed = 1; n->steps_timed = steps; }
    return MC_OK;
  }
  const int k = 2 * n->launches_timed + (begin ? 0 : 1);
  if (k >= kLaunchEvents) return MC_OK;
  HIP_TRY(hipEventRecord(n->ev_launch[(size_t)k], n->stream));
  if (!begin) { ++n->launches_timed; n->steps_timed += steps; }
  return MC_OK;
}

// Enqueues `steps` steps (no synchronization).  Steps are replayed from a
// graph of steps_per_graph steps where possible (0: never).  `call_events`:
// the caller has just recorded ev0 and records ev1 right after, so a call
// that is one launch is timed by those.
int enqueue_steps(mc_net* n, int64_t steps, bool call_events = false) {
  int rc;
  int64_t left = steps;
  bool drained = false;
  while (left > 0) {
    int64_t room = n->cap_steps - n->steps_since_drain;
    if (room <= 0) {
      if ((rc = drain(n)) != MC_OK) return rc;
      room = n->cap_steps;
      drained = true;
    }
    int64_t chunk = std::min(left, room);
    const int S = n->launch.steps_per_graph;
    if (S > 0 && chunk >= S) {
      if ((rc = build_graph(n)) != MC_OK) return rc;
      const int64_t reps = chunk / S;
      const bool whole = call_events && !drained && reps == 1 && S == steps;
      for (int64_t k = 0; k < reps; ++k) {
        if ((rc = launch_event(n, true, S, whole)) != MC_OK) return rc;
        HIP_TRY(hipGraphLaunch(n->graph, n->stream));
        if ((rc = launch_event(n, false, S, whole)) != MC_OK) return rc;
      }
      chunk = reps * S;
    } else {
      chunk = std::min<int64_t>(chunk, 1 << 20);
      // stream events around the launch, unless the call's own bracket it
      // (events that the dispatch itself timestamps cost ~17 us per launch)
      const bool whole = call_events && !drained && chunk == steps;
      if ((rc = launch_event(n, true, chunk, whole)) != MC_OK) return rc;
      HIP_TRY(enqueue_direct(n, (int)chunk, n->stream));
      if ((rc = launch_event(n, false, chunk, whole)) != MC_OK) return rc;
    }
    n->steps_since_drain += chunk;
    n->step += chunk;
    left -= chunk;
  }
  return MC_OK;
}

int upload_network(mc_net* n) {
  HostNet& h = n->h;
  int rc;
  // padded layout
  n->inst_off_pad.assign((size_t)h.n_inst + 1, 0);
  for (int b = 0; b < h.n_inst; ++b)
    n->inst_off_pad[b + 1] = n->inst_off_pad[b] + align_up(h.inst_off[b + 1] - h.inst_off[b], 4);
  n->n_pad = n->inst_off_pad[h.n_inst];
  n->n_quads = n->n_pad / 4;
  n->ring_stride = align_up(n->n_pad, 64);
  const int64_t N = h.N, M = h.M, P = n->n_pad;

  std::vector<int64_t> rp((size_t)P + 1);
  std::vector<double> y((size_t)P, 0.0);
  std::vector<uint64_t> qseed((size_t)n->n_quads);
  std::vector<uint32_t> qlocal((size_t)n->n_quads), qpops((size_t)n->n_quads);
  for (int b = 0; b < h.n_inst; ++b) {
    const int64_t d0 = h.inst_off[b], Nb = h.inst_off[b + 1] - d0, p0 = n->inst_off_pad[b];
    const int64_t Pb = n->inst_off_pad[b + 1] - p0;
    for (int64_t k = 0; k < Pb; ++k) {
      rp[p0 + k] = h.row_ptr[d0 + std::min(k, Nb)];
      if (k < Nb) y[p0 + k] = h.y0[d0 + k];
    }
    for (int64_t qq = 0; qq < Pb / 4; ++qq) {
      const int64_t gq = p0 / 4 + qq;
      qseed[gq] = h.inst_seed[b];
      qlocal[gq] = (uint32_t)qq;
      uint32_t pk = 0;
      for (int k = 0; k < 4; ++k) {
        const int64_t loc = 4 * qq + k;
        const uint32_t pop = loc < Nb ? h.pop_of[d0 + loc] : 0xFFu;
        pk |= pop << (8 * k);
      }
      qpops[gq] = pk;
    }
  }
  rp[P] = M;
  std::vector<int32_t> tg(h.tgt);
  for (int b = 0; b < h.n_inst; ++b) {
    const int64_t shift = n->inst_off_pad[b] - h.inst_off[b];
    if (shift == 0) continue;
    for (int64_t e = h.row_ptr[h.inst_off[b]]; e < h.row_ptr[h.inst_off[b + 1]]; ++e) tg[e] += (int32_t)shift;
  }
  (void)N;
  if ((rc = dev_alloc(n->alloc, &n->d_row_ptr, (size_t)P + 1)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_tgt, (size_t)M)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_wq, (size_t)M)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_dly, (size_t)M)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_y, (size_t)P)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_I, (size_t)P)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_r, (size_t)P)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_ring, (size_t)kRingSlots * n->ring_stride)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_qseed, (size_t)n->n_quads)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_qlocal, (size_t)n->n_quads)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_qpops, (size_t)n->n_quads)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_table, h.table.size())) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_step, 1)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_overflow, 1)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_wbad, 1)) != MC_OK) return rc;
  std::vector<int32_t> qinst((size_t)n->n_quads);
  for (int b = 0; b < h.n_inst; ++b)
    for (int64_t qq = n->inst_off_pad[b] / 4; qq < n->inst_off_pad[b + 1] / 4; ++qq) qinst[qq] = b;
  if ((rc = dev_alloc(n->alloc, &n->d_qinst, (size_t)n->n_quads)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_inst_base, (size_t)h.n_inst + 1)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_ilist, (size_t)2 * P)) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &n->d_icnt, (size_t)2 * h.n_inst)) != MC_OK) return rc;
  HIP_TRY(hipMemcpy(n->d_qinst, qinst.data(), sizeof(int32_t) * n->n_quads, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_inst_base, n->inst_off_pad.data(), sizeof(int64_t) * (h.n_inst + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(n->d_icnt, 0, sizeof(int) * 2 * h.n_inst));
  HIP_TRY(hipMemcpy(n->d_row_ptr, rp.data(), sizeof(int64_t) * (P + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_tgt, tg.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_wq, h.wq.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_dly, h.dly.data(), M, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_y, y.data(), sizeof(double) * P, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(n->d_I, 0, sizeof(double) * P));
  HIP_TRY(hipMemset(n->d_r, 0, sizeof(int32_t) * P));
  HIP_TRY(hipMemset(n->d_ring, 0, sizeof(long long) * kRingSlots * n->ring_stride));
  HIP_TRY(hipMemcpy(n->d_qseed, qseed.data(), sizeof(uint64_t) * n->n_quads, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_qlocal, qlocal.data(), sizeof(uint32_t) * n->n_quads, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_qpops, qpops.data(), sizeof(uint32_t) * n->n_quads, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_table, h.table.data(), sizeof(uint64_t) * h.table.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(n->d_step, 0, sizeof(long long)));
  HIP_TRY(hipMemset(n->d_overflow, 0, sizeof(unsigned)));
  HIP_TRY(hipDeviceSynchronize());
  return MC_OK;
}

}  // namespace

// ===========================================================================
// C interface
// ===========================================================================
extern "C" {

int mc_abi_version(void) { return MC_ABI_VERSION; }

const char* mc_last_error(void) { return g_last_error.c_str(); }

const char* mc_strerror(int code) {
  switch (code) {
    case MC_OK: return "ok";
    case MC_ERR_INVALID_ARG: return "invalid argument";
    case MC_ERR_RANGE: return "value out of range";
    case MC_ERR_OOM: return "out of memory";
    case MC_ERR_HIP: return "HIP runtime error";
    case MC_ERR_STATE: return "invalid handle state";
    case MC_ERR_BUFFER_TOO_SMALL: return "buffer too small";
    case MC_ERR_NO_DEVICE: return "no usable gfx950 device";
    case MC_ERR_MISMATCH: return "recomputation did not reproduce the recorded spikes";
    case MC_ERR_TIMEOUT: return "persistent kernel timed out waiting for spike records";
    default: return "unknown error";
  }
}

int mc_build_network(const mc_config* cfg, mc_net** out) {
  if (!out) return set_error(MC_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!cfg) return set_error(MC_ERR_INVALID_ARG, "cfg is NULL");
  std::unique_ptr<mc_net> n;
  try { n.reset(new mc_net()); } catch (...) { return set_error(MC_ERR_OOM, "host allocation failed"); }
  if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr))
    return set_error(MC_ERR_INVALID_ARG, "dev_alloc and dev_free must be given together");
  if (cfg->struct_size == sizeof(mc_config)) {
    n->alloc.fn = cfg->dev_alloc;
    n->alloc.fr = cfg->dev_free;
    n->alloc.ctx = cfg->alloc_ctx;
  }
  std::string err;
  int rc;
  // connections drawn on the device, on request
  std::unique_ptr<ConnBuilder> conn;
  hipStream_t conn_stream = nullptr;
  if ((cfg->flags & MC_FLAG_DEVICE_CONNECT) != 0) {
    if ((cfg->flags & MC_FLAG_HOST_ONLY) != 0)
      return set_error(MC_ERR_INVALID_ARG, "MC_FLAG_DEVICE_CONNECT needs the device (MC_FLAG_HOST_ONLY given)");
    {
      int ndev = 0, dev = 0;
      hipDeviceProp_t prop;
      if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1 || hipGetDevice(&dev) != hipSuccess ||
          hipGetDeviceProperties(&prop, dev) != hipSuccess || std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(MC_ERR_NO_DEVICE, "MC_FLAG_DEVICE_CONNECT: no gfx950 device");
      if (hipStreamCreateWithFlags(&conn_stream, hipStreamNonBlocking) != hipSuccess)
        return set_error(MC_ERR_HIP, "stream creation failed");
      conn.reset(new_device_conn(prop.multiProcessorCount * 8, conn_stream));
    }
  }
  try { rc = build_host(*cfg, n->h, err, conn.get()); } catch (const std::bad_alloc&) { rc = MC_ERR_OOM; err = "host allocation failed"; }
  conn.reset();
  if (conn_stream) (void)hipStreamDestroy(conn_stream);
  if (rc != MC_OK) return set_error(rc, err);
  n->spikes_base.assign((size_t)n->h.n_pops, 0);
  n->host_only = (cfg->flags & MC_FLAG_HOST_ONLY) != 0;
  if (!n->host_only) {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return set_error(MC_ERR_NO_DEVICE, "no HIP device");
    if (hipGetDevice(&n->device) != hipSuccess) return set_error(MC_ERR_NO_DEVICE, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, n->device) != hipSuccess) return set_error(MC_ERR_NO_DEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      return set_error(MC_ERR_NO_DEVICE, std::string("device is ") + prop.gcnArchName + ", library built for gfx950");
    n->n_cu = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, n->device) == hipSuccess && khz > 0) n->wall_khz = khz;
    int optin = 0;
    if (hipDeviceGetAttribute(&optin, hipDeviceAttributeSharedMemPerBlockOptin, n->device) == hipSuccess && optin > 0)
      n->lds_max = optin;
    else
      n->lds_max = (int)prop.sharedMemPerBlock;
    if (cfg->hip_stream) { n->stream = (hipStream_t)cfg->hip_stream; n->own_stream = false; }
    else {
      if (hipStreamCreateWithFlags(&n->stream, hipStreamNonBlocking) != hipSuccess) return set_error(MC_ERR_HIP, "stream creation failed");
      n->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&n->aux, hipStreamNonBlocking) != hipSuccess) {
      release_all(n.get());
      return set_error(MC_ERR_HIP, "stream creation failed");
    }
    rc = upload_network(n.get());
    // pending input lies at most max_delay slots ahead (until an injection or a loaded state)
    n->horizon = std::max(1, n->h.max_delay);
    if (rc == MC_OK && hipEventCreate(&n->ev0) != hipSuccess) rc = set_error(MC_ERR_HIP, "event creation failed");
    if (rc == MC_OK && hipEventCreate(&n->ev1) != hipSuccess) rc = set_error(MC_ERR_HIP, "event creation failed");
    if (rc == MC_OK && hipEventCreate(&n->ev_mid) != hipSuccess) rc = set_error(MC_ERR_HIP, "event creation failed");
    for (int k = 0; rc == MC_OK && k < kLaunchEvents; ++k) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) rc = set_error(MC_ERR_HIP, "event creation failed");
      else n->ev_launch.push_back(e);
    }
    if (rc == MC_OK) {
      mc_launch l{};
      l.struct_size = sizeof(mc_launch);
      l.scheme = MC_SCHEME_STEP_KERNELS;
      l.block = 256;
      l.neurons_per_wg = 256;
      l.steps_per_graph = 1000;
      n->cap_steps = 8192;
      rc = apply_launch(n.get(), l);
    }
    if (rc != MC_OK) { release_all(n.get()); return rc; }
  }
  *out = n.release();
  return MC_OK;
}

void mc_free(mc_net* n) {
  if (!n) return;
  if (!n->host_only) {
    if (n->stream) (void)hipStreamSynchronize(n->stream);
    release_all(n);
  }
  delete n;
}

int mc_simulate(mc_net* n, int64_t steps) {
  if (!device_ready(n)) return set_error(MC_ERR_STATE, "handle is host-only, failed or NULL");
  if (steps < 0) return set_error(MC_ERR_INVALID_ARG, "steps < 0");
  if (n->step + steps > 2147483647LL) return set_error(MC_ERR_RANGE, "step count beyond int32 raster steps");
  HIP_TRY(hipEventRecord(n->ev0, n->stream));
  n->launches_timed = 0;
  n->steps_timed = 0;
  n->whole_call = false;
  int rc = enqueue_steps(n, steps, true);
  if (rc != MC_OK) { n->failed = true; return rc; }
  HIP_TRY(hipEventRecord(n->ev1, n->stream));
  return MC_OK;
}

int mc_simulate_noalloc(mc_net* n, int64_t steps) {
  if (!device_ready(n)) return set_error(MC_ERR_STATE, "handle is host-only, failed or NULL");
  if (steps < 0) return set_error(MC_ERR_INVALID_ARG, "steps < 0");
  if (n->launch.scheme != MC_SCHEME_PERSISTENT_LDS)
    return set_error(MC_ERR_STATE, "mc_simulate_noalloc runs the persistent scheme only (mc_set_launch scheme 1)");
  if (n->pG > kPersistMaxBlock || n->pB > kPersistMaxB)
    return set_error(MC_ERR_RANGE, "persistent shape beyond the scratch (512 workgroups of 512 targets)");
  if (n->step + steps > 2147483647LL) return set_error(MC_ERR_RANGE, "step count beyond int32 raster steps");
  const int64_t room = n->cap_steps - n->steps_since_drain;
  if (steps > room)
    return set_error(MC_ERR_BUFFER_TOO_SMALL, "the raster has room for " + std::to_string(room) +
                                                  " more steps without a drain; call mc_reserve or mc_get_spikes first");
  int cur = -1;
  HIP_TRY(hipGetDevice(&cur));
  if (cur != n->device) return set_error(MC_ERR_INVALID_ARG, "the network's device is not the current device");
  unsigned long long* rec = nullptr;
  int* pub = nullptr;
  HIP_TRY(noalloc_scratch(n->device, &rec, &pub));
  HIP_TRY(hipEventRecord(n->ev0, n->stream));
  n->launches_timed = 0;
  n->steps_timed = 0;
  n->whole_call = false;
  HIP_TRY(launch_clear_records(rec, persist_flag_words(n->pG), n->stream));
  const DevNet p = n->dev();
  PersistArgs a = n->persist();
  a.flags = rec;
  a.pub = pub;
  int rc;
  for (int64_t left = steps; left > 0;) {
    const int chunk = (int)std::min<int64_t>(left, 1 << 20);
    if ((rc = launch_event(n, true, chunk)) != MC_OK) return rc;
    HIP_TRY(launch_persist(p, a, chunk, n->launch.block, n->stream));
    if ((rc = launch_event(n, false, chunk)) != MC_OK) return rc;
    left -= chunk;
  }
  n->steps_since_drain += steps;
  n->step += steps;
  HIP_TRY(hipEventRecord(n->ev1, n->stream));
  return MC_OK;
}

int mc_last_kernel_ms(mc_net* n, double* ms_out, int64_t* launches_out, int64_t* steps_out) {
  if (!device_ready(n) || !ms_out || !launches_out || !steps_out) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL output");
  HIP_TRY(hipEventSynchronize(n->ev1));
  double total = 0.0;
  for (int k = 0; k < n->launches_timed; ++k) {
    float ms = 0;
    if (n->whole_call) HIP_TRY(hipEventElapsedTime(&ms, n->ev0, n->ev1));
    else HIP_TRY(hipEventElapsedTime(&ms, n->ev_launch[(size_t)2 * k], n->ev_launch[(size_t)2 * k + 1]));
    total += ms;
  }
  *ms_out = total;
  *launches_out = n->launches_timed;
  *steps_out = n->steps_timed;
  return MC_OK;
}

int mc_last_simulate_ms(mc_net* n, double* ms_out) {
  if (!device_ready(n) || !ms_out) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL output");
  HIP_TRY(hipEventSynchronize(n->ev1));
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, n->ev0, n->ev1));
  *ms_out = ms;
  return MC_OK;
}

int mc_reserve(mc_net* n, int64_t steps) {
  if (!device_ready(n)) return set_error(MC_ERR_STATE, "handle is host-only, failed or NULL");
  if (steps < 1 || steps > 2000000) return set_error(MC_ERR_INVALID_ARG, "steps out of [1, 2e6]");
  if (n->cap_steps - n->steps_since_drain >= steps) return MC_OK;
  return setup_recording(n, std::max(steps, n->cap_steps));
}

int mc_get_spikes(mc_net* n, int64_t b, int64_t e, int32_t* st, int32_t* id, int64_t capacity, int64_t* count_out) {
  if (!device_ready(n) || !count_out) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL count_out");
  int rc = drain(n);
  if (rc != MC_OK) return rc;
  auto lo = std::lower_bound(n->r_step.begin(), n->r_step.end(), (int32_t)std::max<int64_t>(std::min<int64_t>(b, 2147483647LL), -1));
  auto hi = std::lower_bound(n->r_step.begin(), n->r_step.end(), (int32_t)std::max<int64_t>(std::min<int64_t>(e, 2147483647LL), -1));
  if (e <= b) hi = lo;
  const int64_t cnt = hi - lo;
  *count_out = cnt;
  if (cnt > capacity) return set_error(MC_ERR_BUFFER_TOO_SMALL, "spike buffer too small");
  if (cnt > 0 && (!st || !id)) return set_error(MC_ERR_INVALID_ARG, "NULL output arrays");
  const size_t o = lo - n->r_step.begin();
  if (cnt) {
    std::copy(n->r_step.begin() + o, n->r_step.begin() + o + cnt, st);
    std::copy(n->r_id.begin() + o, n->r_id.begin() + o + cnt, id);
  }
  return MC_OK;
}

int mc_get_sizes(mc_net* n, int64_t* N, int64_t* M, int32_t* ni) {
  if (!usable(n)) return set_error(MC_ERR_STATE, "bad handle");
  if (N) *N = n->h.N;
  if (M) *M = n->h.M;
  if (ni) *ni = n->h.n_inst;
  return MC_OK;
}

int mc_get_instance_offsets(mc_net* n, int64_t* off) {
  if (!usable(n) || !off) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  std::memcpy(off, n->h.inst_off.data(), sizeof(int64_t) * n->h.inst_off.size());
  return MC_OK;
}

int mc_get_pop_offsets(mc_net* n, int32_t b, int64_t* off) {
  if (!usable(n) || !off || b < 0 || b >= n->h.n_inst) return set_error(MC_ERR_INVALID_ARG, "bad handle, instance or NULL");
  std::memcpy(off, n->h.pop_off.data() + (size_t)b * (n->h.n_pops + 1), sizeof(int64_t) * (n->h.n_pops + 1));
  return MC_OK;
}

int mc_get_synapses(mc_net* n, int64_t* rp, int32_t* tg, int32_t* w, uint8_t* d) {
  if (!usable(n)) return set_error(MC_ERR_STATE, "bad handle");
  const HostNet& h = n->h;
  if (rp) std::memcpy(rp, h.row_ptr.data(), sizeof(int64_t) * (h.N + 1));
  if (tg) std::memcpy(tg, h.tgt.data(), sizeof(int32_t) * h.M);
  if (w) std::memcpy(w, h.wq.data(), sizeof(int32_t) * h.M);
  if (d) std::memcpy(d, h.dly.data(), (size_t)h.M);
  return MC_OK;
}

int mc_get_propagators(mc_net* n, double* p) {
  if (!usable(n) || !p) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  p[0] = n->h.P11; p[1] = n->h.P21; p[2] = n->h.P22; p[3] = n->h.P20;
  return MC_OK;
}

int mc_get_drive_tables(mc_net* n, uint64_t* t) {
  if (!usable(n) || !t) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  std::memcpy(t, n->h.table.data(), sizeof(uint64_t) * n->h.table.size());
  return MC_OK;
}

int mc_get_state(mc_net* n, double* y, double* I, int32_t* r) {
  if (!device_ready(n)) return set_error(MC_ERR_STATE, "handle is host-only, failed or NULL");
  HIP_TRY(hipStreamSynchronize(n->stream));
  const int64_t P = n->n_pad;
  std::vector<double> hy((size_t)P), hI((size_t)P);
  std::vector<int32_t> hr((size_t)P);
  HIP_TRY(hipMemcpy(hy.data(), n->d_y, sizeof(double) * P, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hI.data(), n->d_I, sizeof(double) * P, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hr.data(), n->d_r, sizeof(int32_t) * P, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < n->h.N; ++i) {
    const int64_t pi = n->pad_of(i);
    if (y) y[i] = hy[pi];
    if (I) I[i] = hI[pi];
    if (r) r[i] = hr[pi];
  }
  return MC_OK;
}

int mc_set_state(mc_net* n, const double* y, const double* I, const int32_t* r) {
  if (!device_ready(n) || !y || !I || !r) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  HIP_TRY(hipStreamSynchronize(n->stream));
  const int64_t P = n->n_pad;
  std::vector<double> hy((size_t)P, 0.0), hI((size_t)P, 0.0);
  std::vector<int32_t> hr((size_t)P, 0);
  for (int64_t i = 0; i < n->h.N; ++i) {
    const int64_t pi = n->pad_of(i);
    if (r[i] < 0 || r[i] > 255) return set_error(MC_ERR_RANGE, "refractory count outside [0, 255]");
    hy[pi] = y[i]; hI[pi] = I[i]; hr[pi] = r[i];
  }
  HIP_TRY(hipMemcpy(n->d_y, hy.data(), sizeof(double) * P, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_I, hI.data(), sizeof(double) * P, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(n->d_r, hr.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice));
  return MC_OK;
}

int mc_get_ring(mc_net* n, int64_t depth, int64_t* pending) {
  if (!device_ready(n) || !pending) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  if (depth < 0 || depth > kRingSlots) return set_error(MC_ERR_INVALID_ARG, "depth outside [0, 128]");
  HIP_TRY(hipStreamSynchronize(n->stream));
  std::vector<long long> slot((size_t)n->ring_stride);
  for (int64_t k = 0; k < depth; ++k) {
    const int64_t s = (n->step + k) & kRingMask;
    HIP_TRY(hipMemcpy(slot.data(), n->d_ring + s * n->ring_stride, sizeof(long long) * n->ring_stride, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n->h.N; ++i) pending[k * n->h.N + i] = slot[n->pad_of(i)];
  }
  return MC_OK;
}

int mc_inject(mc_net* n, int64_t k, int64_t neuron, int64_t value) {
  if (!device_ready(n)) return set_error(MC_ERR_STATE, "handle is host-only, failed or NULL");
  if (k < 0 || k >= kRingSlots - 1 || neuron < 0 || neuron >= n->h.N) return set_error(MC_ERR_INVALID_ARG, "k or neuron out of range");
  const int64_t s = (n->step + k) & kRingMask;
  HIP_TRY(launch_inject(n->d_ring, s * n->ring_stride + n->pad_of(neuron), value, n->stream));
  n->horizon = std::max(n->horizon, (int)k + 1);
  return MC_OK;
}

int mc_get_counters(mc_net* n, mc_counters* c) {
  if (!usable(n) || !c) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  std::memset(c, 0, sizeof(*c));
  c->step = n->step;
  if (n->host_only) return MC_OK;
  HIP_TRY(hipStreamSynchronize(n->stream));
  std::vector<unsigned long long> ev((size_t)n->n_wg), sp((size_t)n->n_wg * n->h.n_pops);
  HIP_TRY(hipMemcpy(ev.data(), n->d_wg_events, sizeof(unsigned long long) * ev.size(), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(sp.data(), n->d_wg_spikes, sizeof(unsigned long long) * sp.size(), hipMemcpyDeviceToHost));
  c->events = n->events_base;
  for (auto v : ev) c->events += (int64_t)v;
  for (int a = 0; a < n->h.n_pops; ++a) {
    int64_t s = n->spikes_base[a];
    for (int g = 0; g < n->n_wg; ++g) s += (int64_t)sp[(size_t)g * n->h.n_pops + a];
    c->spikes_per_pop[a] = s;
    c->spikes += s;
  }
  return MC_OK;
}

int mc_set_launch(mc_net* n, const mc_launch* l) {
  if (!device_ready(n) || !l) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  return apply_launch(n, *l);
}

int mc_get_launch(mc_net* n, mc_launch* l) {
  if (!device_ready(n) || !l) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  *l = n->launch;
  return MC_OK;
}

int mc_stream(mc_net* n, void** s) {
  if (!device_ready(n) || !s) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  *s = (void*)n->stream;
  return MC_OK;
}

// Replaces every weight (mode 0: from pA values; 1/2: one gradient step):
// a check pass first, so that a rejected update leaves the store unchanged;
// then the store, the persistent scheme's near-table copies of the delay-1/2
// weights and the host copy.
static int update_weights(mc_net* n, const void* src, int mode, double eta) {
  HIP_TRY(hipMemsetAsync(n->d_wbad, 0, sizeof(unsigned), n->stream));
  HIP_TRY(launch_weights(n->d_wq, src, mode, eta, n->h.M, n->d_wbad, true, n->stream));
  unsigned bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, n->d_wbad, sizeof(unsigned), hipMemcpyDeviceToHost, n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  if (bad) return set_error(MC_ERR_RANGE, "a new weight is not finite or does not fit int32 in units of 2^-16 pA "
                                          "(|w| < 32768 pA); the store is unchanged");
  HIP_TRY(launch_weights(n->d_wq, src, mode, eta, n->h.M, n->d_wbad, false, n->stream));
  if (n->launch.scheme == MC_SCHEME_PERSISTENT_LDS && n->pG > 0 && n->d_ne)
    // the near table holds copies of the delay-1/2 weights
    HIP_TRY(launch_near_fill(n->d_tgt, n->d_wq, n->d_dly, n->d_blk, n->d_bstart, n->n_pad, n->pG, n->d_nb, n->d_ne,
                             n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  HIP_TRY(hipMemcpy(n->h.wq.data(), n->d_wq, sizeof(int32_t) * n->h.M, hipMemcpyDeviceToHost));
  return MC_OK;
}

int mc_set_weights(mc_net* n, const double* w_dev) {
  if (!device_ready(n) || !w_dev) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  return update_weights(n, w_dev, 0, 0.0);
}

int mc_apply_gradient(mc_net* n, const void* grad_dev, int32_t grad_dtype, double eta) {
  if (!device_ready(n) || !grad_dev) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL gradient");
  if (grad_dtype != MC_GRAD_F64 && grad_dtype != MC_GRAD_F32) return set_error(MC_ERR_INVALID_ARG, "unknown grad_dtype");
  if (!std::isfinite(eta)) return set_error(MC_ERR_INVALID_ARG, "eta is not finite");
  return update_weights(n, grad_dev, grad_dtype == MC_GRAD_F64 ? 1 : 2, eta);
}

// Blob: header, y/I/r (padded), ring (all slots), counters.
struct BlobHeader {
  uint64_t magic;
  int64_t n_pad, ring_stride, step, events;
  int64_t spikes[kMaxPops];
};
static const uint64_t kBlobMagic = 0x6d635f7374617431ULL;

int mc_save_state(mc_net* n, void* blob, size_t capacity, size_t* used) {
  if (!device_ready(n) || !used) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  const int64_t P = n->n_pad;
  const size_t need = sizeof(BlobHeader) + P * (sizeof(double) * 2 + sizeof(int32_t)) + sizeof(long long) * kRingSlots * n->ring_stride;
  *used = need;
  if (!blob || capacity < need) return set_error(MC_ERR_BUFFER_TOO_SMALL, "state blob too small");
  mc_counters c;
  int rc = mc_get_counters(n, &c);
  if (rc != MC_OK) return rc;
  BlobHeader hd{};
  hd.magic = kBlobMagic; hd.n_pad = P; hd.ring_stride = n->ring_stride; hd.step = n->step; hd.events = c.events;
  for (int a = 0; a < n->h.n_pops; ++a) hd.spikes[a] = c.spikes_per_pop[a];
  char* o = (char*)blob;
  std::memcpy(o, &hd, sizeof(hd)); o += sizeof(hd);
  HIP_TRY(hipMemcpy(o, n->d_y, sizeof(double) * P, hipMemcpyDeviceToHost)); o += sizeof(double) * P;
  HIP_TRY(hipMemcpy(o, n->d_I, sizeof(double) * P, hipMemcpyDeviceToHost)); o += sizeof(double) * P;
  HIP_TRY(hipMemcpy(o, n->d_r, sizeof(int32_t) * P, hipMemcpyDeviceToHost)); o += sizeof(int32_t) * P;
  HIP_TRY(hipMemcpy(o, n->d_ring, sizeof(long long) * kRingSlots * n->ring_stride, hipMemcpyDeviceToHost));
  return MC_OK;
}

int mc_load_state(mc_net* n, const void* blob, size_t size) {
  if (!device_ready(n) || !blob) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  if (size < sizeof(BlobHeader)) return set_error(MC_ERR_INVALID_ARG, "blob too small");
  BlobHeader hd;
  std::memcpy(&hd, blob, sizeof(hd));
  const int64_t P = n->n_pad;
  const size_t need = sizeof(BlobHeader) + P * (sizeof(double) * 2 + sizeof(int32_t)) + sizeof(long long) * kRingSlots * n->ring_stride;
  if (hd.magic != kBlobMagic || hd.n_pad != P || hd.ring_stride != n->ring_stride || size < need)
    return set_error(MC_ERR_INVALID_ARG, "blob does not belong to this network");
  int rc = drain(n);
  if (rc != MC_OK) return rc;
  const char* o = (const char*)blob + sizeof(hd);
  HIP_TRY(hipMemcpy(n->d_y, o, sizeof(double) * P, hipMemcpyHostToDevice)); o += sizeof(double) * P;
  HIP_TRY(hipMemcpy(n->d_I, o, sizeof(double) * P, hipMemcpyHostToDevice)); o += sizeof(double) * P;
  HIP_TRY(hipMemcpy(n->d_r, o, sizeof(int32_t) * P, hipMemcpyHostToDevice)); o += sizeof(int32_t) * P;
  HIP_TRY(hipMemcpy(n->d_ring, o, sizeof(long long) * kRingSlots * n->ring_stride, hipMemcpyHostToDevice));
  // horizon: one past the last slot ahead of the restored step that holds input
  {
    const long long* ring = reinterpret_cast<const long long*>(o);
    int hz = 1;
    for (int m = kRingSlots - 2; m >= 1 && hz == 1; --m) {
      const long long* slot = ring + (size_t)((hd.step + m) & kRingMask) * n->ring_stride;
      for (int64_t k = 0; k < n->ring_stride; ++k)
        if (slot[k] != 0) { hz = m + 1; break; }
    }
    n->horizon = std::max(hz, std::max(1, n->h.max_delay));
  }
  long long st = hd.step;
  HIP_TRY(hipMemcpy(n->d_step, &st, sizeof(long long), hipMemcpyHostToDevice));
  n->step = hd.step;
  // counters: base = saved totals, device accumulators cleared
  HIP_TRY(hipMemset(n->d_wg_events, 0, sizeof(unsigned long long) * n->n_wg));
  HIP_TRY(hipMemset(n->d_wg_spikes, 0, sizeof(unsigned long long) * n->n_wg * n->h.n_pops));
  n->events_base = hd.events;
  for (int a = 0; a < n->h.n_pops; ++a) n->spikes_base[a] = hd.spikes[a];
  // recorded spikes at or after the restored step are dropped
  auto cut = std::lower_bound(n->r_step.begin(), n->r_step.end(), (int32_t)hd.step);
  const size_t keep = cut - n->r_step.begin();
  n->r_step.resize(keep);
  n->r_id.resize(keep);
  HIP_TRY(hipDeviceSynchronize());
  return MC_OK;
}

int mc_profile_phases(mc_net* n, int64_t steps, double* us) {
  if (!device_ready(n) || !us) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  if (n->launch.scheme != MC_SCHEME_PERSISTENT_LDS && n->launch.scheme != MC_SCHEME_PERSISTENT_BUCKETS)
    return set_error(MC_ERR_STATE, "phase timing needs a persistent scheme");
  if (steps < 1 || n->step + steps > 2147483647LL) return set_error(MC_ERR_INVALID_ARG, "steps out of range");
  int rc;
  const int G = n->launch.scheme == MC_SCHEME_PERSISTENT_LDS ? n->pG : n->own_blocks;
  dev_free(n->alloc, n->d_phase);
  if ((rc = dev_alloc(n->alloc, &n->d_phase, (size_t)G * 8)) != MC_OK) return rc;
  HIP_TRY(hipMemsetAsync(n->d_phase, 0, sizeof(unsigned long long) * G * 8, n->stream));
  // direct launches: a captured graph would carry the timing-off arguments
  if (n->graph) { (void)hipGraphExecDestroy(n->graph); n->graph = nullptr; }
  const int spg = n->launch.steps_per_graph;
  n->launch.steps_per_graph = 0;
  n->phase_on = true;
  n->launches_timed = 0;
  n->steps_timed = 0;
  n->whole_call = false;
  rc = enqueue_steps(n, steps);
  n->phase_on = false;
  n->launch.steps_per_graph = spg;
  if (rc != MC_OK) return rc;
  HIP_TRY(hipStreamSynchronize(n->stream));
  std::vector<unsigned long long> h((size_t)G * 8);
  HIP_TRY(hipMemcpy(h.data(), n->d_phase, sizeof(unsigned long long) * h.size(), hipMemcpyDeviceToHost));
  int khz = 100000;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, n->device) != hipSuccess || khz <= 0) khz = 100000;
  const double tick_us = 1e3 / (double)khz;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int g = 0; g < G; ++g)
    for (int k = 0; k < 7; ++k) acc[k] += (double)h[(size_t)g * 8 + k];
  const double norm = tick_us / ((double)G * (double)steps);
  n->phase_wg.assign((size_t)G * 8, 0.0);
  for (size_t k = 0; k < h.size(); ++k) n->phase_wg[k] = (k % 8 == 7) ? 0.0 : (double)h[k] * tick_us / (double)steps;
  us[5] = 0;
  for (int k = 0; k < 5; ++k) { us[k] = acc[k] * norm; us[5] += us[k]; }
  us[6] = acc[5] * norm;   // drive + pending delivery of wavefront 0 while waiting
  us[7] = acc[6] * norm;   // polling of the first poller thread
  return MC_OK;
}

int mc_get_phase_table(mc_net* n, double* out, int64_t capacity, int32_t* workgroups_out) {
  if (!usable(n) || !workgroups_out) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  const int64_t G = (int64_t)n->phase_wg.size() / 8;
  *workgroups_out = (int32_t)G;
  if (!out || capacity < 8 * G) return G ? set_error(MC_ERR_BUFFER_TOO_SMALL, "phase table buffer too small") : MC_OK;
  std::memcpy(out, n->phase_wg.data(), sizeof(double) * 8 * G);
  return MC_OK;
}

int mc_replay_delivery(mc_net* n, int64_t b, int64_t e, int64_t* ring_out, int64_t ring_cap, double* ms_out,
                       int64_t* events_out) {
  if (!device_ready(n)) return set_error(MC_ERR_STATE, "handle is host-only, failed or NULL");
  if (b < 0 || e <= b || e > n->step) return set_error(MC_ERR_INVALID_ARG, "step range must lie in [0, current step)");
  int rc = drain(n);
  if (rc != MC_OK) return rc;
  const int64_t slots = (e - b) + 101;
  const int64_t N = n->h.N;
  if (ring_out && ring_cap < slots * N) return set_error(MC_ERR_BUFFER_TOO_SMALL, "replay ring buffer too small");
  auto lo = std::lower_bound(n->r_step.begin(), n->r_step.end(), (int32_t)b);
  auto hi = std::lower_bound(n->r_step.begin(), n->r_step.end(), (int32_t)e);
  const size_t o0 = lo - n->r_step.begin(), cnt = hi - lo;
  std::vector<int2> sp(cnt);
  std::vector<long long> first(cnt + 1, 0);
  int64_t events = 0;
  for (size_t k = 0; k < cnt; ++k) {
    const int64_t dense = n->r_id[o0 + k];
    const int64_t len = n->h.row_ptr[dense + 1] - n->h.row_ptr[dense];
    sp[k] = make_int2(n->r_step[o0 + k], (int)n->pad_of(dense));
    first[k + 1] = first[k] + (len + kReplayChunkHost - 1) / kReplayChunkHost;
    events += len;
  }
  int2* d_sp = nullptr;
  long long* d_first = nullptr;
  long long* d_ring = nullptr;
  if ((rc = dev_alloc(n->alloc, &d_sp, std::max<size_t>(cnt, 1))) != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &d_first, cnt + 1)) != MC_OK) { dev_free(n->alloc, d_sp); return rc; }
  if ((rc = dev_alloc(n->alloc, &d_ring, (size_t)slots * n->ring_stride)) != MC_OK) { dev_free(n->alloc, d_sp); dev_free(n->alloc, d_first); return rc; }
  hipError_t err = hipSuccess;
  if (cnt) err = hipMemcpy(d_sp, sp.data(), sizeof(int2) * cnt, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemcpy(d_first, first.data(), sizeof(long long) * (cnt + 1), hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemsetAsync(d_ring, 0, sizeof(long long) * slots * n->ring_stride, n->stream);
  if (err == hipSuccess) err = hipEventRecord(n->ev0, n->stream);
  if (err == hipSuccess && cnt)
    err = launch_replay(d_sp, d_first, (int)cnt, first[cnt], n->d_row_ptr, n->d_tgt, n->d_wq, n->d_dly, d_ring,
                        n->ring_stride, b, n->n_cu * 8, n->stream);
  if (err == hipSuccess) err = hipEventRecord(n->ev1, n->stream);
  if (err == hipSuccess) err = hipEventSynchronize(n->ev1);
  float ms = 0;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, n->ev0, n->ev1);
  if (err == hipSuccess && ring_out) {
    std::vector<long long> slot((size_t)n->ring_stride);
    for (int64_t k = 0; k < slots && err == hipSuccess; ++k) {
      err = hipMemcpy(slot.data(), d_ring + k * n->ring_stride, sizeof(long long) * n->ring_stride, hipMemcpyDeviceToHost);
      for (int64_t i = 0; i < N; ++i) ring_out[k * N + i] = slot[n->pad_of(i)];
    }
  }
  dev_free(n->alloc, d_sp); dev_free(n->alloc, d_first); dev_free(n->alloc, d_ring);
  if (err != hipSuccess) return set_error(MC_ERR_HIP, std::string("replay: ") + hipGetErrorString(err));
  if (ms_out) *ms_out = ms;
  if (events_out) *events_out = events;
  return MC_OK;
}

int mc_atomic_rate(mc_net* n, int64_t entries, double* gops) {
  if (!device_ready(n) || !gops) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  if (entries < 1 || entries > ((int64_t)1 << 32)) return set_error(MC_ERR_INVALID_ARG, "entries out of [1, 2^32]");
  unsigned long long* t = nullptr;
  int rc = dev_alloc(n->alloc, &t, (size_t)entries);
  if (rc != MC_OK) return rc;
  const int grid = n->n_cu * 8;
  const long long per_thread = 256;
  hipError_t err = hipMemsetAsync(t, 0, sizeof(unsigned long long) * entries, n->stream);
  if (err == hipSuccess) err = launch_atomic_rate(t, entries, per_thread, grid, n->stream);   // warm-up
  if (err == hipSuccess) err = hipEventRecord(n->ev0, n->stream);
  if (err == hipSuccess) err = launch_atomic_rate(t, entries, per_thread, grid, n->stream);
  if (err == hipSuccess) err = hipEventRecord(n->ev1, n->stream);
  if (err == hipSuccess) err = hipEventSynchronize(n->ev1);
  float ms = 0;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, n->ev0, n->ev1);
  dev_free(n->alloc, t);
  if (err != hipSuccess) return set_error(MC_ERR_HIP, std::string("atomic rate: ") + hipGetErrorString(err));
  *gops = (double)grid * 256.0 * per_thread / (ms * 1e-3) / 1e9;
  return MC_OK;
}

int mc_probe_stream(mc_net* n, int64_t bytes, double* gbs) {
  if (!device_ready(n) || !gbs) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  if (bytes < (1 << 20) || bytes > ((int64_t)1 << 40)) return set_error(MC_ERR_INVALID_ARG, "bytes out of [1 MiB, 1 TiB]");
  bytes &= ~(int64_t)15;
  unsigned char* buf = nullptr;
  unsigned long long* sink = nullptr;
  int rc = dev_alloc(n->alloc, &buf, (size_t)bytes);
  if (rc != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &sink, 1)) != MC_OK) { dev_free(n->alloc, buf); return rc; }
  const int grid = n->n_cu * 8;
  hipError_t err = hipMemsetAsync(buf, 0x11, (size_t)bytes, n->stream);
  if (err == hipSuccess) err = launch_stream_read(buf, bytes, sink, grid, n->stream);   // warm-up
  if (err == hipSuccess) err = hipEventRecord(n->ev0, n->stream);
  if (err == hipSuccess) err = launch_stream_read(buf, bytes, sink, grid, n->stream);
  if (err == hipSuccess) err = hipEventRecord(n->ev1, n->stream);
  if (err == hipSuccess) err = hipEventSynchronize(n->ev1);
  float ms = 0;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, n->ev0, n->ev1);
  dev_free(n->alloc, buf);
  dev_free(n->alloc, sink);
  if (err != hipSuccess) return set_error(MC_ERR_HIP, std::string("stream probe: ") + hipGetErrorString(err));
  *gbs = (double)bytes / (ms * 1e-3) / 1e9;
  return MC_OK;
}

int mc_probe_atomics(mc_net* n, int64_t slots, int32_t pattern, double* gops) {
  if (!device_ready(n) || !gops) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  if (slots < 1 || slots > 100000) return set_error(MC_ERR_INVALID_ARG, "slots out of [1, 1e5]");
  if (pattern != 0 && pattern != 1) return set_error(MC_ERR_INVALID_ARG, "pattern must be 0 or 1");
  // 1024 quantiles of the store's delay histogram, and its mean out-degree
  if (n->dq.empty()) {
    std::vector<int64_t> hist(kRingSlots, 0);
    for (uint8_t d : n->h.dly) hist[d]++;
    n->dq.assign(1024, 1);
    const double M = (double)std::max<int64_t>(1, n->h.M);
    int64_t cum = 0;
    int d = 0;
    for (int k = 0; k < 1024; ++k) {
      const double q = (k + 0.5) / 1024.0 * M;
      while (d < kRingSlots - 1 && (double)(cum + hist[d]) <= q) cum += hist[d++];
      n->dq[k] = (unsigned char)std::max(1, d);
    }
  }
  const double deg = (double)n->h.M / (double)std::max<int64_t>(1, n->h.N);
  const int gap = (int)std::max(1.0, std::min(1e6, std::round((double)n->h.N / std::max(1.0, deg))));
  unsigned long long* t = nullptr;
  unsigned char* dq = nullptr;
  int rc = dev_alloc(n->alloc, &t, (size_t)slots * n->ring_stride);
  if (rc != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &dq, 1024)) != MC_OK) { dev_free(n->alloc, t); return rc; }
  const int grid = n->n_cu * 8;
  const long long items = 1 << 19;            // 2^27 events per launch
  hipError_t err = hipMemcpy(dq, n->dq.data(), 1024, hipMemcpyHostToDevice);
  if (err == hipSuccess) err = hipMemsetAsync(t, 0, sizeof(unsigned long long) * slots * n->ring_stride, n->stream);
  if (err == hipSuccess)
    err = launch_atomic_slots(t, slots, n->ring_stride, n->n_pad, items, pattern, gap, dq, grid, n->stream);
  // the fastest of three timed launches: the rate the memory system reaches
  float ms = 0;
  for (int rep = 0; rep < 3 && err == hipSuccess; ++rep) {
    float one = 0;
    err = hipEventRecord(n->ev0, n->stream);
    if (err == hipSuccess)
      err = launch_atomic_slots(t, slots, n->ring_stride, n->n_pad, items, pattern, gap, dq, grid, n->stream);
    if (err == hipSuccess) err = hipEventRecord(n->ev1, n->stream);
    if (err == hipSuccess) err = hipEventSynchronize(n->ev1);
    if (err == hipSuccess) err = hipEventElapsedTime(&one, n->ev0, n->ev1);
    if (err == hipSuccess && (rep == 0 || one < ms)) ms = one;
  }
  dev_free(n->alloc, t);
  dev_free(n->alloc, dq);
  if (err != hipSuccess) return set_error(MC_ERR_HIP, std::string("atomic probe: ") + hipGetErrorString(err));
  *gops = (double)items * 256.0 / (ms * 1e-3) / 1e9;
  return MC_OK;
}

int mc_probe_exchange(mc_net* n, int64_t steps, double* us) {
  if (!device_ready(n) || !us) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL");
  if (n->launch.scheme != MC_SCHEME_PERSISTENT_LDS) return set_error(MC_ERR_STATE, "the exchange probe takes the persistent scheme's shape");
  if (steps < 1 || steps > 10000000) return set_error(MC_ERR_INVALID_ARG, "steps out of [1, 1e7]");
  unsigned long long* flags = nullptr;
  unsigned* err_word = nullptr;
  int rc = dev_alloc(n->alloc, &flags, persist_flag_words(n->pG));
  if (rc != MC_OK) return rc;
  if ((rc = dev_alloc(n->alloc, &err_word, 1)) != MC_OK) { dev_free(n->alloc, flags); return rc; }
  const long long wait = (long long)n->wall_khz * 1000 * kWaitSeconds;
  hipError_t err = hipMemsetAsync(flags, 0, sizeof(unsigned long long) * persist_flag_words(n->pG), n->stream);
  if (err == hipSuccess) err = hipMemsetAsync(err_word, 0, sizeof(unsigned), n->stream);
  if (err == hipSuccess) err = launch_exchange_probe(flags, n->pG, n->launch.block, std::min<int64_t>(steps, 1000), wait, err_word, n->stream);
  if (err == hipSuccess) err = hipEventRecord(n->ev0, n->stream);
  if (err == hipSuccess) err = launch_exchange_probe(flags, n->pG, n->launch.block, steps, wait, err_word, n->stream);
  if (err == hipSuccess) err = hipEventRecord(n->ev1, n->stream);
  if (err == hipSuccess) err = hipEventSynchronize(n->ev1);
  float ms = 0;
  unsigned bad = 0;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, n->ev0, n->ev1);
  if (err == hipSuccess) err = hipMemcpy(&bad, err_word, sizeof(unsigned), hipMemcpyDeviceToHost);
  dev_free(n->alloc, flags);
  dev_free(n->alloc, err_word);
  if (err != hipSuccess) return set_error(MC_ERR_HIP, std::string("exchange probe: ") + hipGetErrorString(err));
  if (bad) return set_error(MC_ERR_TIMEOUT, "exchange probe: a workgroup's record never arrived");
  *us = (double)ms * 1e3 / (double)steps;
  return MC_OK;
}

// Key of the autotuner cache: the network's shape and the device.
static std::string tune_key(mc_net* n) {
  uint64_t h = 1469598103934665603ULL;   // FNV-1a over the shape's integers
  auto mix = [&](uint64_t v) {
    for (int k = 0; k < 8; ++k) { h ^= (v >> (8 * k)) & 0xFFu; h *= 1099511628211ULL; }
  };
  // sizes, and the synapse count to an eighth of an octave (about 9 %), so
  // that networks drawn with other seeds share the entry
  mix((uint64_t)n->h.N); mix((uint64_t)n->h.n_inst); mix((uint64_t)n->h.n_pops);
  for (int64_t v : n->h.pop_off) mix((uint64_t)v);
  mix((uint64_t)std::llround(8.0 * std::log2((double)std::max<int64_t>(n->h.M, 1))));
  hipDeviceProp_t prop;
  std::string dev = "unknown";
  if (hipGetDeviceProperties(&prop, n->device) == hipSuccess) {
    dev = prop.gcnArchName;
    for (char& c : dev) if (c == ' ' || c == ':') c = '_';
    dev += "_cu" + std::to_string(prop.multiProcessorCount);
  }
  char buf[32];
  std::snprintf(buf, sizeof(buf), "%016llx", (unsigned long long)h);
  return std::string(buf) + "_" + dev;
}

// The stored choice for `key` (the last line that names it), if any.
static bool tune_cache_read(const char* path, const std::string& key, mc_launch* l) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char k[256];
  int sc, b, npw, spg, rpw;
  double ms;
  bool found = false;
  while (std::fscanf(f, "%255s %d %d %d %d %d %lf", k, &sc, &b, &npw, &spg, &rpw, &ms) == 7) {
    if (key == k) {
      *l = mc_launch{sizeof(mc_launch), sc, b, npw, spg, rpw};
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

static void tune_cache_write(const char* path, const std::string& key, const mc_launch& l, double ms) {
  FILE* f = std::fopen(path, "a");
  if (!f) return;   // an unwritable cache only costs the next run its tuning
  std::fprintf(f, "%s %d %d %d %d %d %.6f\n", key.c_str(), l.scheme, l.block, l.neurons_per_wg, l.steps_per_graph,
               l.rows_per_wave, ms);
  std::fclose(f);
}

// Autotuner: times candidate launch shapes from a saved copy of the current
// state and keeps the fastest.  Every candidate computes the same bits
// (integer input sums, fixed floating-point order), so the choice only
// affects speed; state, counters and the recorded raster are restored.  The
// target-owner scheme is not a candidate: it lost to the step kernels or the
// persistent kernel on every workload measured (a chain of dependent memory
// round trips per step costs more than the atomics it saves).
int mc_tune(mc_net* n, int64_t steps, mc_launch* best) {
  if (!device_ready(n)) return set_error(MC_ERR_STATE, "handle is host-only, failed or NULL");
  if (steps < 1 || steps > 100000) return set_error(MC_ERR_INVALID_ARG, "steps out of [1, 1e5]");
  if (n->step + 2 * steps + 1000 > 2147483647LL) return set_error(MC_ERR_RANGE, "step count beyond int32 raster steps");
  const char* cache = std::getenv("MC_TUNE_CACHE");
  const std::string key = cache && *cache ? tune_key(n) : std::string();
  mc_launch cached{};
  if (!key.empty() && tune_cache_read(cache, key, &cached) && validate_launch(n, cached) == MC_OK &&
      apply_launch(n, cached) == MC_OK) {
    if (best) *best = cached;
    return MC_OK;
  }
  size_t need = 0;
  mc_save_state(n, nullptr, 0, &need);
  std::vector<char> blob;
  try { blob.resize(need); } catch (...) { return set_error(MC_ERR_OOM, "host allocation of the tuning checkpoint failed"); }
  int rc = mc_save_state(n, blob.data(), blob.size(), &need);
  if (rc != MC_OK) return rc;
  const mc_launch original = n->launch;
  const int spg = (int)std::min<int64_t>(steps, 1000);
  // persistent launches of 10,000 steps: the per-launch prologue and
  // epilogue (LDS window in and out) amortise over 1 s of model time
  const int kPersistSteps = 10000;
  const mc_launch cands[] = {
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_LDS, 512, 0, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_LDS, 256, 0, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_LDS, 512, 256, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_LDS, 512, 512, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_LDS, 256, 128, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_BUCKETS, 192, 0, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_BUCKETS, 256, 0, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_BUCKETS, 512, 0, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_PERSISTENT_BUCKETS, 128, 0, kPersistSteps, 0},
      {sizeof(mc_launch), MC_SCHEME_STEP_KERNELS, 256, 256, spg, 0},
      {sizeof(mc_launch), MC_SCHEME_STEP_KERNELS, 256, 256, spg, 1},
      {sizeof(mc_launch), MC_SCHEME_STEP_KERNELS, 256, 1024, spg, 0},
      {sizeof(mc_launch), MC_SCHEME_STEP_KERNELS, 512, 512, spg, 0},
      {sizeof(mc_launch), MC_SCHEME_STEP_KERNELS, 512, 512, spg, 1},
      {sizeof(mc_launch), MC_SCHEME_STEP_KERNELS, 128, 128, spg, 0},
      {sizeof(mc_launch), MC_SCHEME_STEP_KERNELS, 128, 128, spg, 1},
  };
  double best_ms = 1e300;
  mc_launch chosen = original;
  for (const mc_launch& c : cands) {
    if (apply_launch(n, c) != MC_OK) continue;          // shape does not fit this network
    const int64_t warm = c.steps_per_graph > 0 ? std::min<int64_t>(steps, c.steps_per_graph) : std::min<int64_t>(steps, 100);
    if ((rc = mc_reserve(n, warm + steps)) != MC_OK) return rc;
    if ((rc = mc_load_state(n, blob.data(), blob.size())) != MC_OK) return rc;
    if ((rc = enqueue_steps(n, warm)) != MC_OK) return rc;   // warm-up (graph capture, caches)
    HIP_TRY(hipEventRecord(n->ev0, n->stream));
    if ((rc = enqueue_steps(n, steps)) != MC_OK) return rc;
    HIP_TRY(hipEventRecord(n->ev1, n->stream));
    HIP_TRY(hipEventSynchronize(n->ev1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, n->ev0, n->ev1));
    if (ms < best_ms) { best_ms = ms; chosen = c; }
  }
  if ((rc = apply_launch(n, chosen)) != MC_OK) return rc;
  if ((rc = mc_load_state(n, blob.data(), blob.size())) != MC_OK) return rc;
  if (!key.empty() && best_ms < 1e300) tune_cache_write(cache, key, chosen, best_ms / (double)steps);
  if (best) *best = chosen;
  return MC_OK;
}

int mc_get_persist_shape(mc_net* n, int32_t* G, int32_t* B, int32_t* DL) {
  if (!device_ready(n) || !G || !B || !DL) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL output");
  const bool on = n->launch.scheme == MC_SCHEME_PERSISTENT_LDS;
  const bool bk = n->launch.scheme == MC_SCHEME_PERSISTENT_BUCKETS;
  *G = on ? n->pG : bk ? n->own_blocks : 0;
  *B = on ? n->pB : bk ? n->wg_neurons : 0;
  *DL = on ? n->pDL : 0;
  return MC_OK;
}

// Largest input record an adjoint makes by default (8 B per neuron-step).
constexpr double kRecordBudget = 16.0 * 1024 * 1024 * 1024;

int mc_adjoint(mc_net* n, const mc_adjoint_config* a, void* grad, double* loss) {
  if (!device_ready(n)) return set_error(MC_ERR_STATE, "handle is host-only, failed or NULL");
  if (!a || !grad || !loss) return set_error(MC_ERR_INVALID_ARG, "NULL config, gradient or loss pointer");
  if (a->struct_size != sizeof(mc_adjoint_config)) return set_error(MC_ERR_INVALID_ARG, "mc_adjoint_config.struct_size mismatch");
  const int64_t S = a->window_steps, K = a->ckpt_every;
  if (S < 1 || S > 1000000) return set_error(MC_ERR_INVALID_ARG, "window_steps out of [1, 1e6]");
  if (K < 1 || K > 4096) return set_error(MC_ERR_INVALID_ARG, "ckpt_every out of [1, 4096]");
  if (a->grad_dtype != MC_GRAD_F64 && a->grad_dtype != MC_GRAD_F32) return set_error(MC_ERR_INVALID_ARG, "unknown grad_dtype");
  if (a->input_mode != MC_ADJ_INPUT_AUTO && a->input_mode != MC_ADJ_INPUT_RECORD && a->input_mode != MC_ADJ_INPUT_REPLAY)
    return set_error(MC_ERR_INVALID_ARG, "unknown input_mode");
  if (n->step + S > 2147483647LL) return set_error(MC_ERR_RANGE, "step count beyond int32 raster steps");
  const bool fp32 = a->grad_dtype == MC_GRAD_F32;
  const int64_t n0 = n->step;
  const int64_t nseg = (S + K - 1) / K;
  const int64_t st = n->ring_stride;
  const int64_t M = n->h.M;
  const int64_t Kc = std::min(K, S);
  int R = 1;
  while (R < Kc + 101) R <<= 1;
  int rc;
  AdjBuffers B(n->alloc);
  double *ck_y = nullptr, *ck_I = nullptr;
  int32_t* ck_r = nullptr;
  long long* ck_ring = nullptr;
  long long* xrec = nullptr;
  const size_t ring_elems = (size_t)kRingSlots * st;
  const bool record = a->input_mode == MC_ADJ_INPUT_RECORD ||
                      (a->input_mode == MC_ADJ_INPUT_AUTO && (double)S * (double)st * 8.0 <= kRecordBudget);
  if ((rc = B.alloc(&ck_y, (size_t)nseg * st)) != MC_OK) return rc;
  if ((rc = B.alloc(&ck_I, (size_t)nseg * st)) != MC_OK) return rc;
  if ((rc = B.alloc(&ck_r, (size_t)nseg * st)) != MC_OK) return rc;
  if (record) {
    if ((rc = B.alloc(&xrec, (size_t)S * st)) != MC_OK) return rc;
  } else {
    if ((rc = B.alloc(&ck_ring, (size_t)nseg * ring_elems)) != MC_OK) return rc;
  }
  // reverse-pass buffers, allocated and cleared before the forward so that
  // the reverse pass can start as soon as the forward ends
  long long* xseg = nullptr;
  double *rec_y = nullptr, *li_ring = nullptr, *carry = nullptr, *loss_part = nullptr;
  uint8_t* rec_t = nullptr;
  unsigned long long* seg_count = nullptr;
  unsigned* mismatch = nullptr;
  if (!record && (rc = B.alloc(&xseg, (size_t)(Kc + 101) * st)) != MC_OK) return rc;
  if ((rc = B.alloc(&rec_y, (size_t)Kc * st)) != MC_OK) return rc;
  if ((rc = B.alloc(&rec_t, (size_t)Kc * st)) != MC_OK) return rc;
  if ((rc = B.alloc(&li_ring, (size_t)R * st)) != MC_OK) return rc;
  if ((rc = B.alloc(&carry, (size_t)3 * st)) != MC_OK) return rc;
  if ((rc = B.alloc(&seg_count, (size_t)nseg)) != MC_OK) return rc;
  if ((rc = B.alloc(&mismatch, 1)) != MC_OK) return rc;
  loss_part = carry + 2 * st;
  HIP_TRY(hipMemsetAsync(carry, 0, sizeof(double) * 3 * st, n->stream));
  HIP_TRY(hipMemsetAsync(seg_count, 0, sizeof(unsigned long long) * nseg, n->stream));
  HIP_TRY(hipMemsetAsync(mismatch, 0, sizeof(unsigned), n->stream));
  HIP_TRY(hipMemsetAsync(grad, 0, (fp32 ? sizeof(float) : sizeof(double)) * (size_t)M, n->stream));

  // forward (direct launches: a captured graph would carry the record-off
  // arguments).  Record mode: the whole window at once, the update kernels
  // storing the input record and the checkpoints.  Replay mode: checkpoint
  // (state and ring), then K steps, per segment.
  HIP_TRY(hipEventRecord(n->ev0, n->stream));
  const int spg = n->launch.steps_per_graph;
  if (record) {
    n->launch.steps_per_graph = 0;
    n->d_xrec = xrec; n->xrec_step0 = n0; n->xrec_steps = S;
    n->d_ck_y = ck_y; n->d_ck_I = ck_I; n->d_ck_r = ck_r;
    n->ck_step0 = n0; n->ck_every = K; n->ck_count = nseg;
    if ((rc = enqueue_steps(n, S)) != MC_OK) n->failed = true;
  }
  for (int64_t k = 0; !record && k < nseg && rc == MC_OK; ++k) {
    const int64_t len = std::min(K, S - k * K);
    hipError_t e = hipMemcpyAsync(ck_y + k * st, n->d_y, sizeof(double) * n->n_pad, hipMemcpyDeviceToDevice, n->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ck_I + k * st, n->d_I, sizeof(double) * n->n_pad, hipMemcpyDeviceToDevice, n->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ck_r + k * st, n->d_r, sizeof(int32_t) * n->n_pad, hipMemcpyDeviceToDevice, n->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ck_ring + k * ring_elems, n->d_ring, sizeof(long long) * ring_elems, hipMemcpyDeviceToDevice,
                         n->stream);
    if (e != hipSuccess) rc = set_error(MC_ERR_HIP, std::string("checkpoint copy: ") + hipGetErrorString(e));
    else if ((rc = enqueue_steps(n, len)) != MC_OK) n->failed = true;
  }
  n->d_xrec = nullptr; n->xrec_step0 = 0; n->xrec_steps = 0;
  n->d_ck_y = nullptr; n->d_ck_I = nullptr; n->d_ck_r = nullptr;
  n->ck_step0 = 0; n->ck_every = 1; n->ck_count = 0;
  n->launch.steps_per_graph = spg;
  if (rc != MC_OK) return rc;
  HIP_TRY(hipEventRecord(n->ev_mid, n->stream));

  const DevNet p = n->dev();
  const double c = 2.0 / ((double)n->h.N * (double)S);
  const double ystar = a->v_target_mV - n->h.e_l;
  const int grid = n->n_cu * 8;
  auto seg_args = [&](int64_t k) {
    const int64_t s0 = n0 + k * K, len = std::min(K, S - k * K);
    AdjSeg sg{};
    sg.a = s0; sg.len = (int)len; sg.R = R; sg.c = c; sg.ystar = ystar;
    sg.ck_y = ck_y + k * st; sg.ck_I = ck_I + k * st; sg.ck_r = ck_r + k * st;
    sg.xseg = record ? xrec + (size_t)(s0 - n0) * st : xseg;
    sg.x_has_drive = record ? 1 : 0;
    sg.rec_y = rec_y; sg.rec_t = rec_t; sg.li_ring = li_ring;
    sg.carry_ly = carry; sg.carry_li = carry + st; sg.loss_part = loss_part; sg.spike_count = seg_count + k;
    return sg;
  };
  // the last segment's recomputation needs only checkpoints and the input
  // record: it runs while the raster is read back
  if (record) HIP_TRY(launch_adj_segment(p, seg_args(nseg - 1), n->stream));
  if ((rc = drain(n, n->ev_mid)) != MC_OK) return rc;

  // recorded spikes of the window (dense ids sorted by step, id)
  const auto lo = std::lower_bound(n->r_step.begin(), n->r_step.end(), (int32_t)n0) - n->r_step.begin();
  const auto hi = std::lower_bound(n->r_step.begin(), n->r_step.end(), (int32_t)(n0 + S)) - n->r_step.begin();
  auto spikes_in = [&](int64_t b, int64_t e, size_t* first, size_t* count) {
    b = std::max(b, n0); e = std::min(e, n0 + S);
    if (e <= b) { *first = (size_t)lo; *count = 0; return; }
    const auto x = std::lower_bound(n->r_step.begin() + lo, n->r_step.begin() + hi, (int32_t)b) - n->r_step.begin();
    const auto y = std::lower_bound(n->r_step.begin() + lo, n->r_step.begin() + hi, (int32_t)e) - n->r_step.begin();
    *first = (size_t)x; *count = (size_t)(y - x);
  };
  // Per segment, three work lists: the spikes to deliver into the replayed
  // input (t in [a, a+len-1); replay mode only), to verify (t in [a, a+len))
  // and to gather (t in [a-2, a+len-2), t <= n0+S-3).  Their sizes are known
  // from the raster; each is built on the host just before its segment, into
  // pinned staging, and copied with the segment's kernels on the stream, so
  // the host builds segment k-1's lists while the device runs segment k.
  struct SegLists {
    size_t dl_f, dl_c, vf_f, vf_c, ga_f, ga_c;   // raster ranges
    size_t o_dl, o_first, o_vf, o_srcs, o_gfirst, o_times;   // byte offsets in the staging / device arena
  };
  std::vector<SegLists> L((size_t)nseg);
  size_t bytes = 0;
  auto take = [&](size_t n_bytes) { const size_t o = bytes; bytes += (n_bytes + 15) & ~(size_t)15; return o; };
  for (int64_t k = 0; k < nseg; ++k) {
    const int64_t s0 = n0 + k * K, len = std::min(K, S - k * K);
    SegLists& q = L[(size_t)k];
    q.dl_f = q.dl_c = 0;
    if (!record) spikes_in(s0, s0 + len - 1, &q.dl_f, &q.dl_c);
    spikes_in(s0, s0 + len, &q.vf_f, &q.vf_c);
    spikes_in(s0 - 2, std::min(s0 + len - 2, n0 + S - 2), &q.ga_f, &q.ga_c);
    q.o_dl = take(sizeof(int2) * q.dl_c);
    q.o_first = take(sizeof(long long) * (q.dl_c + 1));
    q.o_vf = take(sizeof(int2) * q.vf_c);
    q.o_srcs = take(sizeof(int4) * q.ga_c);
    q.o_gfirst = take(sizeof(long long) * (q.ga_c + 1));
    q.o_times = take(sizeof(int) * q.ga_c);
  }
  unsigned char* d_lists = nullptr;
  if ((rc = B.alloc(&d_lists, bytes)) != MC_OK) return rc;
  if (n->stage_bytes < bytes) {
    if (n->h_stage) { (void)hipHostFree(n->h_stage); n->h_stage = nullptr; n->stage_bytes = 0; }
    HIP_TRY(hipHostMalloc(&n->h_stage, bytes, hipHostMallocDefault));
    n->stage_bytes = bytes;
  }
  unsigned char* h = static_cast<unsigned char*>(n->h_stage);
  std::vector<unsigned long long> want_count((size_t)nseg);
  std::vector<unsigned long long> keys;
  for (int64_t k = nseg - 1; k >= 0; --k) {
    const int64_t s0 = n0 + k * K, len = std::min(K, S - k * K);
    const SegLists& q = L[(size_t)k];
    // replay mode: the spikes whose delivery rebuilds the segment's input
    long long dl_chunks = 0;
    if (!record) {
      int2* dl = reinterpret_cast<int2*>(h + q.o_dl);
      long long* first = reinterpret_cast<long long*>(h + q.o_first);
      for (size_t z = 0; z < q.dl_c; ++z) {
        const int64_t dense = n->r_id[q.dl_f + z];
        const int64_t rl = n->h.row_ptr[dense + 1] - n->h.row_ptr[dense];
        dl[z] = make_int2(n->r_step[q.dl_f + z], (int)n->pad_of(dense));
        first[z] = dl_chunks;
        dl_chunks += (rl + kReplayChunkHost - 1) / kReplayChunkHost;
      }
      first[q.dl_c] = dl_chunks;
    }
    int2* vf = reinterpret_cast<int2*>(h + q.o_vf);
    for (size_t z = 0; z < q.vf_c; ++z) vf[z] = make_int2(n->r_step[q.vf_f + z], (int)n->pad_of(n->r_id[q.vf_f + z]));
    want_count[(size_t)k] = q.vf_c;
    // dl, first and vf lie before the gather lists in the arena: one copy
    HIP_TRY(hipMemcpyAsync(d_lists + q.o_dl, h + q.o_dl, q.o_srcs - q.o_dl, hipMemcpyHostToDevice, n->stream));
    if (!record) {
      HIP_TRY(launch_adj_seed(xseg, ck_ring + k * ring_elems, st, s0, (int)(len + 101), n->stream));
      if (q.dl_c)
        HIP_TRY(launch_replay(reinterpret_cast<const int2*>(d_lists + q.o_dl),
                              reinterpret_cast<const long long*>(d_lists + q.o_first), (int)q.dl_c, dl_chunks,
                              n->d_row_ptr, n->d_tgt, n->d_wq, n->d_dly, xseg, st, s0, grid, n->stream));
    }
    if (!(record && k == nseg - 1)) HIP_TRY(launch_adj_segment(p, seg_args(k), n->stream));
    HIP_TRY(launch_adj_verify(reinterpret_cast<const int2*>(d_lists + q.o_vf), (int)q.vf_c, rec_t, st, s0, mismatch,
                              n->stream));
    // gather: group by source (ascending), times decreasing; per source its chunk range
    keys.resize(q.ga_c);
    for (size_t z = 0; z < q.ga_c; ++z)
      keys[z] = (unsigned long long)(uint32_t)n->r_id[q.ga_f + z] << 32 | (uint32_t)(0x7FFFFFFF - n->r_step[q.ga_f + z]);
    std::sort(keys.begin(), keys.end());
    int4* srcs = reinterpret_cast<int4*>(h + q.o_srcs);
    long long* gfirst = reinterpret_cast<long long*>(h + q.o_gfirst);
    int* times = reinterpret_cast<int*>(h + q.o_times);
    long long chunks = 0;
    int nsrc = 0;
    for (size_t z = 0; z < q.ga_c;) {
      size_t e = z;
      const uint32_t src = (uint32_t)(keys[z] >> 32);
      while (e < q.ga_c && (uint32_t)(keys[e] >> 32) == src) ++e;
      const int64_t rl = n->h.row_ptr[src + 1] - n->h.row_ptr[src];
      for (size_t y = z; y < e; ++y) times[y] = 0x7FFFFFFF - (int)(uint32_t)(keys[y] & 0xFFFFFFFFu);
      srcs[nsrc] = make_int4((int)n->pad_of(src), (int)z, (int)(e - z), 0);
      gfirst[nsrc] = chunks;
      chunks += (rl + kGatherChunkHost - 1) / kGatherChunkHost;
      ++nsrc;
      z = e;
    }
    gfirst[nsrc] = chunks;
    if (nsrc == 0) continue;
    HIP_TRY(hipMemcpyAsync(d_lists + q.o_srcs, h + q.o_srcs, sizeof(int4) * nsrc, hipMemcpyHostToDevice, n->stream));
    HIP_TRY(hipMemcpyAsync(d_lists + q.o_gfirst, h + q.o_gfirst, sizeof(long long) * (nsrc + 1), hipMemcpyHostToDevice,
                           n->stream));
    HIP_TRY(hipMemcpyAsync(d_lists + q.o_times, h + q.o_times, sizeof(int) * q.ga_c, hipMemcpyHostToDevice, n->stream));
    HIP_TRY(launch_adj_gather(reinterpret_cast<const int4*>(d_lists + q.o_srcs),
                              reinterpret_cast<const long long*>(d_lists + q.o_gfirst), nsrc, chunks,
                              reinterpret_cast<const int*>(d_lists + q.o_times), n->d_row_ptr, n->d_tgt, n->d_dly,
                              li_ring, st, R, n0 + S - 1, grad, fp32, grid, n->stream));
  }
  HIP_TRY(hipEventRecord(n->ev1, n->stream));
  HIP_TRY(hipStreamSynchronize(n->stream));
  float fwd_ms = 0, rev_ms = 0;
  HIP_TRY(hipEventElapsedTime(&fwd_ms, n->ev0, n->ev_mid));
  HIP_TRY(hipEventElapsedTime(&rev_ms, n->ev_mid, n->ev1));
  n->adj_forward_ms = fwd_ms;
  n->adj_reverse_ms = rev_ms;
  unsigned mm = 0;
  std::vector<unsigned long long> got(nseg);
  HIP_TRY(hipMemcpy(&mm, mismatch, sizeof(unsigned), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(got.data(), seg_count, sizeof(unsigned long long) * nseg, hipMemcpyDeviceToHost));
  for (int64_t k = 0; k < nseg && mm == 0; ++k)
    if (got[k] != want_count[k]) mm = 1;
  if (mm) return set_error(MC_ERR_MISMATCH, "recomputed segment does not reproduce the recorded spikes");
  std::vector<double> lp((size_t)st);
  HIP_TRY(hipMemcpy(lp.data(), loss_part, sizeof(double) * st, hipMemcpyDeviceToHost));
  double sum = 0.0;
  for (int64_t i = 0; i < n->n_pad; ++i) sum += lp[i];
  *loss = sum / ((double)n->h.N * (double)S);
  return MC_OK;
}

int mc_last_adjoint_ms(mc_net* n, double* forward_ms, double* reverse_ms) {
  if (!device_ready(n) || !forward_ms || !reverse_ms) return set_error(MC_ERR_INVALID_ARG, "bad handle or NULL output");
  *forward_ms = n->adj_forward_ms;
  *reverse_ms = n->adj_reverse_ms;
  return MC_OK;
}

}  // extern "C"
