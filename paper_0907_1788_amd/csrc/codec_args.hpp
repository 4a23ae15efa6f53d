// Kernel arguments of the encoder and decoder, and the helpers that move V
// lanes of one row between global memory and registers.
#pragma once
#include "field.hpp"

namespace fntrs {

struct EncodeArgs {
  const uint32_t* src;
  uint64_t ld_src, stride_src;
  uint32_t* dst;
  uint64_t ld_dst, stride_dst;
  const uint32_t* tw;        // tw[e] = 3^e
  const uint32_t* twi;       // twi[e] = 3^-e
  uint32_t n, k, lanes;
  int logn, logK;            // transform size K = 2^logK >= k, K <= n
  uint32_t tiles, cosets;    // lane tiles per block, n / K
  uint32_t vec;              // src/dst rows are 16-byte aligned (vector access allowed)
  uint32_t rows_out;         // only rows i < rows_out of dst are written (0: all n)
};

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

struct DecodeArgs {
  const uint32_t* recv;
  uint64_t ld_recv, stride_recv;
  uint32_t* dst;
  uint64_t ld_dst, stride_dst;
  const uint32_t* tw;
  const uint32_t* twi;
  const uint32_t* wfull;    // per position z < n: decoder weight (0 if z is erased)
  const uint32_t* ridx;     // per position z < n: row of z in a compact recv
  const uint32_t* ahat_br;  // FNT_M of A's low part, bit-reversed order, times M^-1
  uint32_t n, k, lanes;
  int logn, logk;
  uint32_t full;            // recv holds n rows indexed by position
  uint32_t tiles, vec;
  uint32_t row0;            // a received row of recv: erased positions read it and discard the value
};

// Work table of the batched path: the jobs of one class (one transform size,
// one kernel configuration) share a persistent launch; job j owns the work
// items [start[j], start[j+1]), numbered as the single-job grid numbers its
// workgroups.
template <class Args>
struct JobTable {
  const Args* jobs;
  const uint32_t* start;    // njobs + 1 ascending entries, start[0] = 0
  uint32_t njobs, total;    // total = start[njobs]
};

}  // namespace fntrs
