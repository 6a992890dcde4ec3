// mc_common.h -- definitions shared by libmc's host builder and its HIP kernels.
//
// Counter-based random numbers: Philox4x64-10 as published by Salmon, Moraes,
// Dror and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11).  A
// block is a pure function of (counter[4], key[2]), so every draw of the
// simulation is addressed by what it is for -- (step, neuron quad) for the
// drive, (source, target) for a connection -- and results are independent of
// thread counts, launch shapes and batching.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define MC_HD __host__ __device__ __forceinline__
#else
#define MC_HD inline
#endif

namespace mc {

// Stream tags (last counter word).
enum : uint64_t { kTagV0 = 1, kTagConn = 2, kTagSrc = 3, kTagW = 4, kTagD = 5, kTagDrive = 6, kTagScale = 7 };

constexpr int kRingSlots = 128;          // input ring depth (power of two)
constexpr int kRingMask = kRingSlots - 1;
constexpr int kMaxPops = 16;
constexpr int kTableLen = 64;            // Poisson inverse-CDF entries per population

struct U64x4 { uint64_t w0, w1, w2, w3; };

MC_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

// Philox4x64 with ten rounds.  Round: the products of counter words 0 and 2
// with the two multipliers; high halves are mixed with the other counter
// words and the round key, low halves pass through.  The key advances by the
// two Weyl constants between rounds.
MC_HD U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t kMulA = 0xD2E7470EE14C6C93ULL, kMulB = 0xCA5A826395121157ULL;
  const uint64_t kWeylA = 0x9E3779B97F4A7C15ULL, kWeylB = 0xBB67AE8584CAA73BULL;
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
#endif
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo_a = kMulA * c0, hi_a = mulhi64(kMulA, c0);
    const uint64_t lo_b = kMulB * c2, hi_b = mulhi64(kMulB, c2);
    const uint64_t n0 = hi_b ^ c1 ^ k0;
    const uint64_t n2 = hi_a ^ c3 ^ k1;
    c0 = n0; c1 = lo_b; c2 = n2; c3 = lo_a;
    k0 += kWeylA; k1 += kWeylB;
  }
  return U64x4{c0, c1, c2, c3};
}

MC_HD uint64_t pick(const U64x4& v, unsigned k) {
  return k == 0 ? v.w0 : k == 1 ? v.w1 : k == 2 ? v.w2 : v.w3;
}

// Uniforms from one 64-bit word.
MC_HD uint32_t hi32(uint64_t w) { return (uint32_t)(w >> 32); }
MC_HD double u01_closed_open(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }        // [0, 1)
MC_HD double u01_open_closed(uint64_t w) { return (double)((w >> 11) + 1) * 0x1p-53; }  // (0, 1]

}  // namespace mc
