// mc_construct.hip -- connections of the pairwise Bernoulli rule and sources
// of the fixed in-degree rule drawn on the device.
//
// Instantiation is untimed (Methods), and for the microcircuit most of it is
// the pair test: every (source, target) pair of an instance is tested against
// its population pair's threshold, about 6e9 tests at full scale.  The test
// is pure integer work on counter-based Philox draws, so the device gives the
// host's result bit for bit: source i connects to target j iff the upper 32
// bits of word j&3 of the block keyed (i, j>>2, 0, CONN) are below
// floor(p * 2^32).  Weights and delays (normal draws through the C library's
// log and cos) stay on the host.
//
// One wavefront per source row: lanes take consecutive quads of targets (one
// Philox block each), so the row's targets come out in ascending order; a
// count pass sizes the rows, a fill pass writes them.
//
// The fixed in-degree rule draws every target's sources with replacement:
// draw m of target j takes the multiply-shift bounded integer (u * N_b) >> 32
// of the upper 32 bits u of word m&3 of the block keyed (j, m>>2, 0, SRC).
// Only these integer draws move to the device; the host sorts them by
// source into rows and draws weights and delays.
#include "mc_build.h"
#include "mc_device.h"

namespace mc {

namespace {

struct BernArgs {
  long long N;
  int n;
  uint64_t seed;
  const long long* off;             // [n+1]
  const uint8_t* pop;               // [N]
  const unsigned long long* thr;    // [n*n], [post][pre]
};

constexpr int kConnBlock = 256;

__device__ __forceinline__ unsigned quad_mask(const BernArgs& a, long long i, long long q, long long j0, long long j1,
                                              uint64_t T) {
  const U64x4 v = philox4x64_10((uint64_t)i, (uint64_t)q, 0, kTagConn, a.seed, 0);
  unsigned m = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long j = 4 * q + k;
    if (j >= j0 && j < j1 && (uint64_t)hi32(pick(v, (unsigned)k)) < T) m |= 1u << k;
  }
  return m;
}

__global__ __launch_bounds__(kConnBlock) void k_bern_count(BernArgs a, long long* counts) {
  const int lane = threadIdx.x & 63;
  const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long i = wave; i < a.N; i += nwaves) {
    const int b = a.pop[i];
    int cnt = 0;
    for (int t = 0; t < a.n; ++t) {
      const uint64_t T = a.thr[t * a.n + b];
      if (T == 0) continue;
      const long long j0 = a.off[t], j1 = a.off[t + 1];
      for (long long q = (j0 >> 2) + lane; q <= ((j1 - 1) >> 2); q += 64) cnt += __popc(quad_mask(a, i, q, j0, j1, T));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
    if (lane == 0) counts[i] = cnt;
  }
}

__global__ __launch_bounds__(kConnBlock) void k_bern_fill(BernArgs a, const long long* row_ptr, long long goff,
                                                          int32_t* tgt) {
  const int lane = threadIdx.x & 63;
  const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long i = wave; i < a.N; i += nwaves) {
    const int b = a.pop[i];
    long long pos = row_ptr[i] - row_ptr[0];
    const long long end = row_ptr[i + 1] - row_ptr[0];   // the count pass made the same draws: pos ends here
    for (int t = 0; t < a.n; ++t) {
      const uint64_t T = a.thr[t * a.n + b];
      if (T == 0) continue;
      const long long j0 = a.off[t], j1 = a.off[t + 1], qend = (j1 - 1) >> 2;
      for (long long q0 = j0 >> 2; q0 <= qend; q0 += 64) {
        const long long q = q0 + lane;
        const unsigned m = (q <= qend) ? quad_mask(a, i, q, j0, j1, T) : 0u;
        const int c = __popc(m);
        int x = c;                                // inclusive prefix over lanes (ascending targets)
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(x, o, 64);
          if (lane >= o) x += y;
        }
        long long w = pos + (x - c);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if ((m & (1u << k)) && w < end) tgt[w++] = (int32_t)(goff + 4 * q + k);
        pos += __shfl(x, 63, 64);
      }
    }
  }
}

// Fixed in-degree sources: one wavefront per target j, lanes on consecutive
// Philox blocks (four draws each); draw m of target j comes from the
// population whose cumulative count K[pop(j)][0..b] first exceeds m.
struct FixedArgs {
  long long N;
  int n;
  uint64_t seed;
  const long long* off;             // [n+1]
  const uint8_t* pop;               // [N]
  const long long* K;               // [n*n], [post][pre]
  const long long* first;           // [N+1]
};

__global__ __launch_bounds__(kConnBlock) void k_fixed_sources(FixedArgs a, int32_t* src) {
  const int lane = threadIdx.x & 63;
  const long long wave = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  const long long nwaves = ((long long)gridDim.x * blockDim.x) >> 6;
  for (long long j = wave; j < a.N; j += nwaves) {
    const int post = a.pop[j];
    const long long kin = a.first[j + 1] - a.first[j];
    for (long long q = lane; 4 * q < kin; q += 64) {
      const U64x4 v = philox4x64_10((uint64_t)j, (uint64_t)q, 0, kTagSrc, a.seed, 0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const long long m = 4 * q + k;
        if (m >= kin) break;
        int b = 0;
        long long cum = a.K[post * a.n];
        while (m >= cum) { ++b; cum += a.K[post * a.n + b]; }
        const uint64_t Nb = (uint64_t)(a.off[b + 1] - a.off[b]);
        src[a.first[j] + m] = (int32_t)(a.off[b] + (long long)(((uint64_t)hi32(pick(v, (unsigned)k)) * Nb) >> 32));
      }
    }
  }
}

template <class T>
hipError_t dalloc(T** p, size_t n) { return hipMalloc((void**)p, (n ? n : 1) * sizeof(T)); }

// Device copies of one plan's small arrays.
struct PlanDev {
  long long* off = nullptr;
  uint8_t* pop = nullptr;
  unsigned long long* thr = nullptr;
  ~PlanDev() { (void)hipFree(off); (void)hipFree(pop); (void)hipFree(thr); }
  hipError_t load(const BernoulliPlan& b, hipStream_t s) {
    hipError_t e = dalloc(&off, (size_t)b.n_pops + 1);
    if (e == hipSuccess) e = dalloc(&pop, (size_t)b.N);
    if (e == hipSuccess) e = dalloc(&thr, (size_t)b.n_pops * b.n_pops);
    if (e == hipSuccess) e = hipMemcpyAsync(off, b.off, sizeof(long long) * (b.n_pops + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(pop, b.pop, (size_t)b.N, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(thr, b.thr, sizeof(unsigned long long) * b.n_pops * b.n_pops, hipMemcpyHostToDevice, s);
    return e;
  }
  BernArgs args(const BernoulliPlan& b) const { return BernArgs{(long long)b.N, b.n_pops, b.seed, off, pop, thr}; }
};

class DeviceConn : public ConnBuilder {
 public:
  DeviceConn(int grid, hipStream_t s) : grid_(grid), s_(s) {}

  int count(const BernoulliPlan& b, int64_t* counts, std::string& err) override {
    PlanDev d;
    long long* dc = nullptr;
    hipError_t e = d.load(b, s_);
    if (e == hipSuccess) e = dalloc(&dc, (size_t)b.N);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_bern_count, dim3(grid_), dim3(kConnBlock), 0, s_, d.args(b), dc);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(counts, dc, sizeof(long long) * b.N, hipMemcpyDeviceToHost, s_);
    if (e == hipSuccess) e = hipStreamSynchronize(s_);
    (void)hipFree(dc);
    return check(e, err);
  }

  int fill(const BernoulliPlan& b, const int64_t* row_ptr_local, int32_t* tgt, std::string& err) override {
    PlanDev d;
    long long* drp = nullptr;
    int32_t* dt = nullptr;
    const long long M = row_ptr_local[b.N] - row_ptr_local[0];
    hipError_t e = d.load(b, s_);
    if (e == hipSuccess) e = dalloc(&drp, (size_t)b.N + 1);
    if (e == hipSuccess) e = dalloc(&dt, (size_t)M);
    if (e == hipSuccess)
      e = hipMemcpyAsync(drp, row_ptr_local, sizeof(long long) * (b.N + 1), hipMemcpyHostToDevice, s_);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_bern_fill, dim3(grid_), dim3(kConnBlock), 0, s_, d.args(b), drp, (long long)b.goff, dt);
      e = hipGetLastError();
    }
    if (e == hipSuccess && M > 0) e = hipMemcpyAsync(tgt, dt, sizeof(int32_t) * M, hipMemcpyDeviceToHost, s_);
    if (e == hipSuccess) e = hipStreamSynchronize(s_);
    (void)hipFree(drp);
    (void)hipFree(dt);
    return check(e, err);
  }

  int sources(const FixedPlan& f, int32_t* src, std::string& err) override {
    const long long Mb = f.first[f.N];
    long long *off = nullptr, *K = nullptr, *first = nullptr;
    uint8_t* pop = nullptr;
    int32_t* ds = nullptr;
    hipError_t e = dalloc(&off, (size_t)f.n_pops + 1);
    if (e == hipSuccess) e = dalloc(&K, (size_t)f.n_pops * f.n_pops);
    if (e == hipSuccess) e = dalloc(&first, (size_t)f.N + 1);
    if (e == hipSuccess) e = dalloc(&pop, (size_t)f.N);
    if (e == hipSuccess) e = dalloc(&ds, (size_t)Mb);
    if (e == hipSuccess) e = hipMemcpyAsync(off, f.off, sizeof(long long) * (f.n_pops + 1), hipMemcpyHostToDevice, s_);
    if (e == hipSuccess)
      e = hipMemcpyAsync(K, f.K, sizeof(long long) * f.n_pops * f.n_pops, hipMemcpyHostToDevice, s_);
    if (e == hipSuccess) e = hipMemcpyAsync(first, f.first, sizeof(long long) * (f.N + 1), hipMemcpyHostToDevice, s_);
    if (e == hipSuccess) e = hipMemcpyAsync(pop, f.pop, (size_t)f.N, hipMemcpyHostToDevice, s_);
    if (e == hipSuccess) {
      const FixedArgs a{(long long)f.N, f.n_pops, f.seed, off, pop, K, first};
      hipLaunchKernelGGL(k_fixed_sources, dim3(grid_), dim3(kConnBlock), 0, s_, a, ds);
      e = hipGetLastError();
    }
    if (e == hipSuccess && Mb > 0) e = hipMemcpyAsync(src, ds, sizeof(int32_t) * Mb, hipMemcpyDeviceToHost, s_);
    if (e == hipSuccess) e = hipStreamSynchronize(s_);
    (void)hipFree(off); (void)hipFree(K); (void)hipFree(first); (void)hipFree(pop); (void)hipFree(ds);
    return check(e, err);
  }

 private:
  static int check(hipError_t e, std::string& err) {
    if (e == hipSuccess) return MC_OK;
    err = std::string("device connection drawing: ") + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? MC_ERR_OOM : MC_ERR_HIP;
  }
  int grid_;
  hipStream_t s_;
};

}  // namespace

ConnBuilder* new_device_conn(int grid, hipStream_t s) { return new DeviceConn(grid, s); }

}  // namespace mc
