// Encoder and decoder kernels: one workgroup owns a tile of T = V*G lanes of
// one codeword block and runs every transform of that block on chip
// (registers + LDS), so each block's data crosses HBM once in each direction.
#pragma once
#include "regfnt.hpp"

namespace fntrs {

constexpr int kCodecThreads = 512;

struct EncodeArgs {
  const uint32_t* src;
  uint64_t ld_src, stride_src;
  uint32_t* dst;
  uint64_t ld_dst, stride_dst;
  const uint32_t* tw;        // tw[e] = 3^e
  uint32_t n, k, lanes;
  int logn, logK;            // transform size K = 2^logK >= k, K <= n
  uint32_t tiles, cosets;    // lane tiles per block, n / K
  uint32_t G;                // lane groups per tile (T = V*G)
  uint32_t vec;              // src/dst rows are 16-byte aligned (vector access allowed)
};

// Moves V lanes of one row between global memory and registers; lanes at or
// beyond `lanes` read as 0 and are not written.
template <int V>
__device__ __forceinline__ void gload(const uint32_t* p, uint32_t lane, uint32_t lanes, bool vec,
                                      uint32_t (&x)[V]) {
  if constexpr (V == 4) {
    if (vec && lane + 4 <= lanes) {
      const uint4 t = *reinterpret_cast<const uint4*>(p);
      x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
      return;
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) x[v] = (lane + v < lanes) ? p[v] : 0u;
}

template <int V>
__device__ __forceinline__ void gstore(uint32_t* p, uint32_t lane, uint32_t lanes, bool vec,
                                       const uint32_t (&x)[V]) {
  if constexpr (V == 4) {
    if (vec && lane + 4 <= lanes) {
      *reinterpret_cast<uint4*>(p) = make_uint4(canon(x[0]), canon(x[1]), canon(x[2]), canon(x[3]));
      return;
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v)
    if (lane + v < lanes) p[v] = canon(x[v]);
}

// Encoder, Sec. II-B: e_i = s(r_n^i).  Output row i = t + (n/K) m is output m
// of FNT_K applied to (s_j r_n^(t j))_j, since r_n^(n/K) = r_K:
//   s(r_n^(t + (n/K) m)) = sum_j (s_j r_n^(t j)) r_K^(m j).
// One workgroup per (lane tile, coset t, block); rows j >= k are the zero
// padding and are never read.
template <int V, int BMAX>
__global__ void __launch_bounds__(kCodecThreads) k_encode(EncodeArgs a) {
  extern __shared__ uint32_t lds[];
  // coset fastest, then lane tile: the workgroups that read the same source
  // lines (all cosets of one tile, then the neighbouring tiles) run together
  uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t t = bid % a.cosets;
  bid /= a.cosets;
  const uint32_t tile = bid % a.tiles;
  const uint64_t blk = bid / a.tiles;
  const uint32_t G = a.G;
  const uint32_t lane0 = tile * (V * G);
  const uint32_t* src = a.src + blk * a.stride_src + lane0;
  uint32_t* dst = a.dst + blk * a.stride_dst + lane0;
  const bool vec = a.vec;
  const int sh = 16 - a.logn;

  auto ld0 = [&](uint32_t pos, uint32_t g, uint32_t (&x)[V]) {
    const uint32_t j = bitrev(pos, a.logK);
    if (j >= a.k) {
#pragma unroll
      for (int v = 0; v < V; ++v) x[v] = 0;
      return;
    }
    gload<V>(src + (uint64_t)j * a.ld_src + g * V, lane0 + g * V, a.lanes, vec, x);
    if (t) {
      const uint32_t w = a.tw[((t * j) & (a.n - 1)) << sh];
#pragma unroll
      for (int v = 0; v < V; ++v) x[v] = fmul(x[v], w);
    }
  };
  auto ldm = [&](uint32_t pos, uint32_t g, uint32_t (&x)[V]) { lds_get<V>(lds, pos * G + g, x); };
  auto stm = [&](uint32_t pos, uint32_t g, const uint32_t (&x)[V]) { lds_put<V>(lds, pos * G + g, x); };
  auto stl = [&](uint32_t pos, uint32_t g, const uint32_t (&x)[V]) {
    const uint64_t row = t + (uint64_t)a.cosets * pos;
    gstore<V>(dst + row * a.ld_dst + g * V, lane0 + g * V, a.lanes, vec, x);
  };
  if (a.logK == 0) {
    // k = 1: every encoded symbol equals s_0 (FNT_1 is the identity).
    for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) {
      uint32_t x[V];
      ld0(0, g, x);
      stl(0, g, x);
    }
    return;
  }
  dit_transform<V, BMAX>(a.logK, G, false, a.tw, false, ld0, ldm, stm, stl);
}

struct DecodeArgs {
  const uint32_t* recv;
  uint64_t ld_recv, stride_recv;
  uint32_t* dst;
  uint64_t ld_dst, stride_dst;
  const uint32_t* tw;
  const uint32_t* wfull;    // per position z < n: decoder weight (0 if z is erased)
  const uint32_t* ridx;     // per position z < n: row of z in a compact recv
  const uint32_t* ahat;     // FNT_2k of A's low part, natural order, times (2k)^-1
  uint32_t n, k, lanes;
  int logn, logk;
  uint32_t full;            // recv holds n rows indexed by position
  uint32_t tiles, G, vec;
};

// Decoder, Sec. II-B steps 4-6, for one (lane tile, block):
//   step 4  n_i = v_i / A'(x_i).  The locator's weight for received position
//           z_i is -r_n^(-z_i) / A'(x_i), so u_z = weight_z * v_z already
//           carries the sign and the index shift of step 5 (0 when z is erased);
//   step 5  S_j = -N'(r^(-j-1)) = sum_z u_z r^(-j z), j < k: one unscaled
//           inverse FNT_n of u (DIT; inputs read from global memory in
//           bit-reversed order);
//   step 6  P = (A S) mod x^k: FNT_2k of (S, 0) times FNT_2k(A mod x^k)/2k,
//           inverse FNT_2k, keep the first k coefficients.
// Between transforms the last pass writes its outputs in bit-reversed order,
// which is the input order of the next DIT transform.  With k = n (nothing
// erased) the weights are n^-1 and the inverse FNT_n alone is the decoder
// (Sec. II-B, erasure-free case).
template <int V, int BMAX>
__global__ void __launch_bounds__(kCodecThreads) k_decode(DecodeArgs a) {
  extern __shared__ uint32_t lds[];
  const uint32_t bid = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t tile = bid % a.tiles;
  const uint64_t blk = bid / a.tiles;
  const uint32_t G = a.G;
  const uint32_t lane0 = tile * (V * G);
  const uint32_t* recv = a.recv + blk * a.stride_recv + lane0;
  uint32_t* dst = a.dst + blk * a.stride_dst + lane0;
  const bool vec = a.vec;
  const uint32_t n = a.n, k = a.k;
  const int log2k = a.logk + 1;

  auto ldg = [&](uint32_t pos, uint32_t g, uint32_t (&x)[V]) {
    const uint32_t z = bitrev(pos, a.logn);
    const uint32_t w = a.wfull[z];
    if (w == 0) {
#pragma unroll
      for (int v = 0; v < V; ++v) x[v] = 0;
      return;
    }
    const uint32_t row = a.full ? z : a.ridx[z];
    gload<V>(recv + (uint64_t)row * a.ld_recv + g * V, lane0 + g * V, a.lanes, vec, x);
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = fmul(x[v], w);
  };
  auto ldl = [&](uint32_t pos, uint32_t g, uint32_t (&x)[V]) { lds_get<V>(lds, pos * G + g, x); };
  auto stl = [&](uint32_t pos, uint32_t g, const uint32_t (&x)[V]) { lds_put<V>(lds, pos * G + g, x); };
  auto stg = [&](uint32_t pos, uint32_t g, const uint32_t (&x)[V]) {
    if (pos < k) gstore<V>(dst + (uint64_t)pos * a.ld_dst + g * V, lane0 + g * V, a.lanes, vec, x);
  };

  if (k == n) {
    if (a.logn == 0) {
      for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) {
        uint32_t x[V];
        ldg(0, g, x);
        stg(0, g, x);
      }
      return;
    }
    dit_transform<V, BMAX>(a.logn, G, true, a.tw, false, ldg, ldl, stl, stg);
    return;
  }
  // step 5: S in bit-reversed order of size 2k (zeros at indices k..2k-1)
  auto st_s = [&](uint32_t m, uint32_t g, const uint32_t (&x)[V]) {
    if (m >= 2 * k) return;
    uint32_t y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) y[v] = m < k ? x[v] : 0u;
    lds_put<V>(lds, bitrev(m, log2k) * G + g, y);
  };
  dit_transform<V, BMAX>(a.logn, G, true, a.tw, true, ldg, ldl, stl, st_s);
  // step 6: FNT_2k(S) * Ahat / 2k, back in bit-reversed order
  auto st_p = [&](uint32_t m, uint32_t g, const uint32_t (&x)[V]) {
    const uint32_t h = a.ahat[m];
    uint32_t y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) y[v] = fmul(canon(x[v]), h);
    lds_put<V>(lds, bitrev(m, log2k) * G + g, y);
  };
  dit_transform<V, BMAX>(log2k, G, false, a.tw, true, ldl, ldl, stl, st_p);
  dit_transform<V, BMAX>(log2k, G, true, a.tw, false, ldl, ldl, stl, stg);
}

}  // namespace fntrs
