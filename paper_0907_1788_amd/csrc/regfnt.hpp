// Register-resident FNT passes over GF(65537) for gfx950.
//
// A transform of size m = 2^logm along the rows of a tile (every lane an
// independent transform, Sec. II-B) runs as a sequence of passes.  A pass
// fuses B radix-2 decimation-in-time stages (the divide-and-conquer FNT of
// Sec. II-A): each thread loads one "item" -- the 2^B positions
// base + c*2^s0, c < 2^B, for V adjacent lanes -- into registers, runs the B
// stages there and stores it back.  Passes read and write a swizzled LDS
// tile; the first pass may read global memory and the last may write it.
// DIT order: position p of the first pass holds input index bitrev(p); the
// last pass leaves output m at position m.
//
// Arithmetic keeps values "semi-canonical": int32 in [-1, 65536], where -1
// stands for 65536.  With p = 2^16 + 1, 2^16 = -1, so a 32-bit word
// hi*2^16 + lo is congruent to lo - hi; the butterfly
//     t = y*w (y made canonical by an unsigned min, w < 65536, product < 2^32)
//     t <- lo(t) - hi(t)               in (-65536, 65536)
//     x' = x + t,  y' = x - t          in [-65536, 131071]
//     x' <- lo16(x') - (x' >> 16)      (signed high half) in [-1, 65536]
// costs one multiply and six adds/logic ops.  Stores to global memory take
// the canonical residue min(x, 65536) (as unsigned, -1 -> 65536).
#pragma once
#include "field.hpp"

namespace fntrs {

__device__ __forceinline__ uint32_t sfold(int32_t a) {
  return (uint32_t)((int32_t)(a & 0xFFFF) - (a >> 16));
}

__device__ __forceinline__ uint32_t canon(uint32_t x) { return min(x, 65536u); }

// Semi-canonical DIT butterfly (x, y) -> (x + w y, x - w y), w in [1, 65535].
__device__ __forceinline__ void bfly(uint32_t& x, uint32_t& y, uint32_t w) {
  const uint32_t yc = min(y, 65536u);
  const uint32_t m = __umul24(yc, w);
  const int32_t t = (int32_t)(m & 0xFFFFu) - (int32_t)(m >> 16);
  const int32_t a = (int32_t)x + t;
  const int32_t b = (int32_t)x - t;
  x = sfold(a);
  y = sfold(b);
}

// Exponent of omega_(2^lg)^j in the table tw[e] = 3^e (inverse root if inv).
__device__ __forceinline__ uint32_t twe(uint32_t j, int lg, bool inv) {
  const uint32_t e = (j << (16 - lg)) & 0xFFFFu;
  return inv ? ((65536u - e) & 0xFFFFu) : e;
}

// LDS tile: position pos, lane group g (V lanes each) at vector index
// u = pos*G + g, XOR-swizzled so that the strided item accesses of the
// passes spread over the banks.
__device__ __forceinline__ uint32_t swz(uint32_t u) { return u ^ ((u >> 4) & 7u); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that consecutive logical ids run on the same XCD:
// neighbouring lane tiles, which share cache lines of every row, then meet
// in one L2 instead of each fetching whole lines from HBM.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nb) {
  const uint32_t xcd = bid & 7u, local = bid >> 3;
  const uint32_t per = nb >> 3, rem = nb & 7u;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <int V>
__device__ __forceinline__ void lds_get(const uint32_t* lds, uint32_t u, uint32_t (&x)[V]) {
  const uint32_t* p = lds + swz(u) * V;
  if constexpr (V == 4) {
    const uint4 t = *reinterpret_cast<const uint4*>(p);
    x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
  } else if constexpr (V == 2) {
    const uint2 t = *reinterpret_cast<const uint2*>(p);
    x[0] = t.x; x[1] = t.y;
  } else {
    x[0] = p[0];
  }
}

template <int V>
__device__ __forceinline__ void lds_put(uint32_t* lds, uint32_t u, const uint32_t (&x)[V]) {
  uint32_t* p = lds + swz(u) * V;
  if constexpr (V == 4) {
    *reinterpret_cast<uint4*>(p) = make_uint4(x[0], x[1], x[2], x[3]);
  } else if constexpr (V == 2) {
    *reinterpret_cast<uint2*>(p) = make_uint2(x[0], x[1]);
  } else {
    p[0] = x[0];
  }
}

// B DIT stages s0 .. s0+B-1 on one item: x[c] is position base + c*2^s0,
// jp = base mod 2^s0.  Stage s0+i pairs c and c + 2^i; the twiddle of the
// pair is omega_(2^(s0+i+1))^(jp + (c mod 2^i) 2^s0).
template <int B, int V>
__device__ __forceinline__ void dit_item(uint32_t (&x)[1 << B][V], int s0, uint32_t jp, bool inv,
                                         const uint32_t* __restrict__ tw) {
#pragma unroll
  for (int i = 0; i < B; ++i) {
    const int half = 1 << i;
    const int lg = s0 + i + 1;
#pragma unroll
    for (int cc = 0; cc < half; ++cc) {
      const uint32_t w = tw[twe(jp + ((uint32_t)cc << s0), lg, inv)];
#pragma unroll
      for (int c0 = 0; c0 < (1 << B); c0 += 2 * half) {
#pragma unroll
        for (int v = 0; v < V; ++v) bfly(x[c0 + cc][v], x[c0 + cc + half][v], w);
      }
    }
  }
}

// One DIT pass over every item of a size-2^logm transform on G lane groups.
// ld(pos, g, x) / st(pos, g, x) move one position of one lane group.
// With `sync`, every thread first loads and transforms its single item, the
// block synchronises, and only then are results stored: needed when the
// store goes to LDS positions that other items still have to read (the
// caller guarantees items <= blockDim.x in that case).
template <int B, int V, class Ld, class St>
__device__ __forceinline__ void dit_pass(int logm, int s0, uint32_t G, bool inv, const uint32_t* __restrict__ tw,
                                         bool sync, Ld&& ld, St&& st) {
  const uint32_t items = (1u << (logm - B)) * G;
  const uint32_t H = 1u << s0;
  if (!sync) {
    for (uint32_t q = threadIdx.x; q < items; q += blockDim.x) {
      const uint32_t g = q % G, it = q / G;
      const uint32_t jp = it & (H - 1);
      const uint32_t base = ((it >> s0) << (s0 + B)) | jp;
      uint32_t x[1 << B][V];
#pragma unroll
      for (int c = 0; c < (1 << B); ++c) ld(base + c * H, g, x[c]);
      dit_item<B, V>(x, s0, jp, inv, tw);
#pragma unroll
      for (int c = 0; c < (1 << B); ++c) st(base + c * H, g, x[c]);
    }
  } else {
    const uint32_t q = threadIdx.x;
    const bool act = q < items;
    const uint32_t g = q % G, it = q / G;
    const uint32_t jp = it & (H - 1);
    const uint32_t base = ((it >> s0) << (s0 + B)) | jp;
    uint32_t x[1 << B][V];
    if (act) {
#pragma unroll
      for (int c = 0; c < (1 << B); ++c) ld(base + c * H, g, x[c]);
      dit_item<B, V>(x, s0, jp, inv, tw);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int c = 0; c < (1 << B); ++c) st(base + c * H, g, x[c]);
    }
  }
}

// Pass plan: radices (B per pass) for a size-2^logm transform.  The last
// pass takes the largest radix min(bmax, logm) (it bounds the item count of
// a synchronised last pass); the remaining stages are split as evenly as
// possible, larger radices later.  Returns the number of passes.
__host__ __device__ __forceinline__ int plan_passes(int logm, int bmax, int (&bs)[8]) {
  if (logm == 0) return 0;
  const int last = logm < bmax ? logm : bmax;
  const int rest = logm - last;
  const int nr = (rest + bmax - 1) / bmax;
  for (int p = 0; p < nr; ++p) bs[p] = rest / nr + (p >= nr - rest % nr ? 1 : 0);
  bs[nr] = last;
  return nr + 1;
}

// Largest radix to plan with: every pass should have at least one item per
// thread (items = G 2^(logm-B) >= threads), at least radix 8, never more
// than BMAX.
__host__ __device__ __forceinline__ int pass_bmax(int logm, uint32_t G, uint32_t threads, int bmax) {
  int lt = 0;
  while ((G << lt) < threads) ++lt;          // log2(threads / G)
  int b = logm - lt;
  const int floor_b = logm < 3 ? logm : 3;   // radix-8 passes at least: idle threads cost less
  if (b < floor_b) b = floor_b;              // than extra round trips through LDS
  if (b > bmax) b = bmax;
  return b;
}

// Runs a whole DIT transform: pass p uses loader (p == 0 ? first : mid) and
// storer (p == last ? last : mid); `sync_last` requests the synchronised
// variant for the last pass.  A barrier separates passes.
template <int V, int BMAX, class LdFirst, class LdMid, class StMid, class StLast>
__device__ __forceinline__ void dit_transform(int logm, uint32_t G, bool inv, const uint32_t* __restrict__ tw,
                                              bool sync_last, LdFirst&& ld0, LdMid&& ldm, StMid&& stm,
                                              StLast&& stl) {
  int bs[8];
  const int np = plan_passes(logm, pass_bmax(logm, G, blockDim.x, BMAX), bs);
  int s0 = 0;
  for (int p = 0; p < np; ++p) {
    const bool first = p == 0, last = p == np - 1;
    const int b = bs[p];
    auto ld = [&](uint32_t pos, uint32_t g, uint32_t (&x)[V]) {
      if (first) ld0(pos, g, x); else ldm(pos, g, x);
    };
    auto st = [&](uint32_t pos, uint32_t g, const uint32_t (&x)[V]) {
      if (last) stl(pos, g, x); else stm(pos, g, x);
    };
    const bool sync = last && sync_last;
    switch (b) {
      case 1: dit_pass<1, V>(logm, s0, G, inv, tw, sync, ld, st); break;
      case 2: dit_pass<2, V>(logm, s0, G, inv, tw, sync, ld, st); break;
      case 3: dit_pass<3, V>(logm, s0, G, inv, tw, sync, ld, st); break;
      case 4: dit_pass<4, V>(logm, s0, G, inv, tw, sync, ld, st); break;
      case 5:
        if constexpr (BMAX >= 5) dit_pass<(BMAX >= 5 ? 5 : 1), V>(logm, s0, G, inv, tw, sync, ld, st);
        break;
      default:
        if constexpr (BMAX >= 6) dit_pass<(BMAX >= 6 ? 6 : 1), V>(logm, s0, G, inv, tw, sync, ld, st);
        break;
    }
    s0 += b;
    __syncthreads();
  }
}

}  // namespace fntrs
