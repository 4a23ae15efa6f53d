// Arithmetic in GF(65537) for gfx950 kernels (Sec. II-A/II-B of Soro & Lacan).
//
// Residues are kept canonical in [0, 65536] as uint32.  Reduction uses the
// Fermat structure of p = 2^16 + 1: 2^16 = -1 (mod p), so a 32-bit word
// hi*2^16 + lo is congruent to lo - hi, which lies in (-2^16, 2^16); one
// conditional add of p makes it canonical.  2^32 = 1 (mod p) handles the one
// product that needs 33 bits (65536 * 65536).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernel_args.hpp"

namespace fntrs {

// Global-memory views of generic pointers.  A pointer that reaches a kernel
// through memory (a job table) rather than as a kernel argument has lost its
// address space, and flat accesses through it count against the LDS counter
// too, so that every wait for an LDS result would also wait for all global
// traffic in flight.  Every global access of the coding kernels goes
// through these views.
#define FNTRS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const FNTRS_GLOBAL T* gptr(const T* p) {
  return (const FNTRS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ FNTRS_GLOBAL T* gptr(T* p) {
  return (FNTRS_GLOBAL T*)p;
}

// 16-byte vector of the global accesses.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// A trivially copyable struct read from global memory word by word.
template <class T>
__device__ __forceinline__ T load_global(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  T v;
  const FNTRS_GLOBAL uint32_t* q = gptr(reinterpret_cast<const uint32_t*>(p));
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (unsigned i = 0; i < sizeof(T) / 4; ++i) d[i] = q[i];
  return v;
}


constexpr uint32_t kP = 65537u;

// a + b mod p for canonical a, b.
__device__ __forceinline__ uint32_t fadd(uint32_t a, uint32_t b) {
  uint32_t s = a + b;
  return min(s, s - kP);            // s < p: s - p wraps above s
}

// a - b mod p for canonical a, b.
__device__ __forceinline__ uint32_t fsub(uint32_t a, uint32_t b) {
  uint32_t d = a + kP - b;          // in [1, 131073]
  return min(d, d - kP);
}

// Fold a 32-bit word m (m < 2^32) to its canonical residue: m = hi*2^16 + lo = lo - hi.
__device__ __forceinline__ uint32_t ffold(uint32_t m) {
  uint32_t t = (m & 0xFFFFu) - (m >> 16);   // wraps when lo < hi
  return min(t, t + kP);
}

// a * w mod p for canonical a and a twiddle w in [0, 65535]: the product is
// below 2^32 and the 24-bit multiplier is exact for both operands.
__device__ __forceinline__ uint32_t fmul_tw(uint32_t a, uint32_t w) {
  return ffold(__umul24(a, w));
}

// a * b mod p for any canonical a, b (the product may be exactly 2^32).
__device__ __forceinline__ uint32_t fmul(uint32_t a, uint32_t b) {
  uint64_t m = (uint64_t)a * b;
  uint32_t lo = (uint32_t)m, hi = (uint32_t)(m >> 32);     // hi is 0 or 1
  uint32_t t = (lo & 0xFFFFu) + hi - (lo >> 16);
  return min(t, t + kP);
}

// x^(p-2) = x^65535 = x^(2^16 - 1): the inverse of a nonzero x (Fermat).
__device__ __forceinline__ uint32_t finv(uint32_t x) {
  uint32_t acc = x, sq = x;
  #pragma unroll
  for (int i = 1; i < 16; ++i) {
    sq = fmul(sq, sq);
    acc = fmul(acc, sq);
  }
  return acc;
}

// Reverse the low `bits` bits of x (bits = 0 gives 0).
__device__ __forceinline__ uint32_t bitrev(uint32_t x, int bits) {
  return bits == 0 ? 0u : (__brev(x) >> (32 - bits));
}

}  // namespace fntrs
