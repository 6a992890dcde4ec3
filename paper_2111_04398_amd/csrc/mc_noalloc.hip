// mc_noalloc.hip -- device scratch of the allocation-free simulation entry
// point (mc_simulate_noalloc).
//
// The persistent kernel exchanges spikes through per-workgroup records and a
// side array for the ids beyond those a record carries.  mc_simulate keeps
// them in memory the library allocates when the launch shape is set; the
// allocation-free entry point takes them from this file-scope array instead,
// sized for the largest persistent shape (512 workgroups of 512 targets).
// Every GPU the library runs on holds its own copy until the process ends.
// Host code must not pass `scratch` itself to a kernel (on the host it is a
// stand-in symbol, not a device address): the device address is looked up
// once per device with hipGetSymbolAddress, with that device current.
#include <mutex>

#include "mc_device.h"

namespace mc {

namespace {

constexpr size_t kScratchRecordWords = (size_t)kPersistMaxBlock * kRecSlots * kPersistFlagStride + kPersistFlagStride;
constexpr size_t kScratchPubInts = (size_t)kPersistMaxBlock * kRecSlots * kPersistMaxB;
constexpr size_t kScratchWords = kScratchRecordWords + kScratchPubInts / 2;

static __device__ __align__(256) unsigned long long scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

__global__ void k_fill_u64(unsigned long long* p, long long n, unsigned long long v) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
    p[k] = v;
}

}  // namespace

size_t noalloc_scratch_bytes() { return sizeof(unsigned long long) * kScratchWords; }
size_t noalloc_record_words() { return kScratchRecordWords; }

// Device address of this device's scratch, looked up on the first call for
// the device (which must be current) and kept: records first, then the side
// array of ids.
hipError_t noalloc_scratch(int device, unsigned long long** records, int** pub) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *records = static_cast<unsigned long long*>(g_scratch_ptr[device]);
  *pub = reinterpret_cast<int*>(*records + kScratchRecordWords);
  return hipSuccess;
}

// Clears `words` record words with a fill kernel (no memset node if the
// caller captures the stream into a graph).
hipError_t launch_clear_records(unsigned long long* records, size_t words, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(64), dim3(256), 0, s, records, (long long)words, 0ull);
  return hipGetLastError();
}

}  // namespace mc
