// Kernel arguments of the encoder and decoder, and the helpers that move V
// lanes of one row between global memory and registers.
#pragma once
#include "field.hpp"
#include "kernel_args.hpp"

namespace fntrs {


// Moves V lanes of one row between global memory and registers.  The
// whole-vector forms make one 16-byte access (V = 4, aligned rows, all V
// lanes present); the part forms read lanes at or beyond `lanes` as 0 and do
// not write them.  Callers pick the form once per item, outside their loop
// over rows, so that each loop is one clean sequence of accesses.
template <int V>
__device__ __forceinline__ void gload_whole(const uint32_t* p, uint32_t (&x)[V]) {
  if constexpr (V == 4) {
    const u32x4 t = *(const FNTRS_GLOBAL u32x4*)gptr(p);
    x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
  } else {
    const FNTRS_GLOBAL uint32_t* q = gptr(p);
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = q[v];
  }
}

template <int V>
__device__ __forceinline__ void gload_part(const uint32_t* p, uint32_t lane, uint32_t lanes, uint32_t (&x)[V]) {
  const FNTRS_GLOBAL uint32_t* q = gptr(p);
#pragma unroll
  for (int v = 0; v < V; ++v) x[v] = (lane + v < lanes) ? q[v] : 0u;
}

template <int V>
__device__ __forceinline__ void gstore_whole(uint32_t* p, const uint32_t (&x)[V]) {
  if constexpr (V == 4) {
    const u32x4 t = {x[0], x[1], x[2], x[3]};
    *(FNTRS_GLOBAL u32x4*)gptr(p) = t;
  } else {
    FNTRS_GLOBAL uint32_t* q = gptr(p);
#pragma unroll
    for (int v = 0; v < V; ++v) q[v] = x[v];
  }
}

template <int V>
__device__ __forceinline__ void gstore_part(uint32_t* p, uint32_t lane, uint32_t lanes, const uint32_t (&x)[V]) {
  FNTRS_GLOBAL uint32_t* q = gptr(p);
#pragma unroll
  for (int v = 0; v < V; ++v)
    if (lane + v < lanes) q[v] = x[v];
}

// Whether the V lanes from `lane` can move as one whole vector.
template <int V>
__device__ __forceinline__ bool whole_vector(uint32_t lane, uint32_t lanes, bool vec) {
  return lane + V <= lanes && (V != 4 || vec);
}



}  // namespace fntrs
