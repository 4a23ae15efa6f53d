// Fused evaluation on a geometric sequence (the chirp of Sec. II-B): the
// cyclic product of length P = 2^LP <= 2^13 of one lane tile of one block
// stays in LDS, so each block crosses HBM once in each direction:
//   DIF FNT_P of u (the coefficients reversed and scaled by a^j q^(-t_j),
//     read from global memory, natural order in, bit-reversed out),
//   times v^ = FNT_P(q^(t_m)) stored in bit-reversed order,
//   inverse DIT FNT_P (bit-reversed in, natural out), of which the middle
//     coefficients L-1 .. L+M-2 are scaled by q^(-t_i) / P and stored.
#pragma once
#include "ct_kernels.hpp"

namespace fntrs {

struct ChirpArgs {
  const uint32_t* c;        // coefficients [block][L][lanes]
  uint64_t ld_c, st_c;
  uint32_t* out;            // values [block][M][lanes]
  uint64_t ld_o, st_o;
  const uint32_t* su;       // a^j q^(-t_j), j < L
  const uint32_t* so;       // q^(-t_i) / P, i < M
  const uint32_t* vhat_br;  // FNT_P(v) in bit-reversed order
  const uint32_t* tw;
  const uint32_t* twi;
  uint32_t L, M, lanes, tiles, vec;
};

namespace ct {

// First DIF pass: position p (natural) holds coefficient L-1-p times its
// scale, zero from p = L on (the padding of the length-P product).
template <int V>
struct ChirpLoad {
  const uint32_t* c;   // block base + lane0
  uint64_t ld;
  const uint32_t* su;
  uint32_t L, lane0, lanes;
  bool vec;
  template <int B, uint32_t H, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int cc = 0; cc < (1 << B); ++cc) {
      const uint32_t p = base + cc * H;
      if (p < L) load_lanes<V, WHOLE>(row_ptr(c, L - 1 - p, ld) + g * V, lane0 + g * V, lanes, x[cc]);
      else
#pragma unroll
        for (int v = 0; v < V; ++v) x[cc][v] = 0;
    }
#pragma unroll
    for (int cc = 0; cc < (1 << B); ++cc) {
      const uint32_t p = base + cc * H;
      const uint32_t w = p < L ? gptr(su)[L - 1 - p] : 0u;
#pragma unroll
      for (int v = 0; v < V; ++v) x[cc][v] = mulc((uint32_t)x[cc][v], w);
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    if (whole_vector<V>(lane0 + g * V, lanes, vec)) rows<B, H, true>(base, g, x);
    else rows<B, H, false>(base, g, x);
  }
};

// Last DIT pass: coefficient m (natural) of the product, kept for
// L-1 <= m < L-1+M as output row m-(L-1), times its scale.
template <int V>
struct ChirpStore {
  uint32_t* out;       // block base + lane0
  uint64_t ld;
  const uint32_t* so;
  uint32_t L, M, lane0, lanes;
  bool vec;
  template <int B, uint32_t H, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int cc = 0; cc < (1 << B); ++cc) {
      const uint32_t m = base + cc * H;
      if (m + 1 < L || m + 1 - L >= M) continue;
      const uint32_t i = m + 1 - L;
      const uint32_t s = gptr(so)[i];
      int32_t y[V];
#pragma unroll
      for (int v = 0; v < V; ++v) y[v] = mulc(canon(x[cc][v]), s);
      store_lanes<V, WHOLE>(out + (uint64_t)i * ld + g * V, lane0 + g * V, lanes, y);
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    if (whole_vector<V>(lane0 + g * V, lanes, vec)) rows<B, H, true>(base, g, x);
    else rows<B, H, false>(base, g, x);
  }
};

// One workgroup per (lane tile, block).
template <int LP, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_chirp(ChirpArgs a) {
  using Gm = Geo<LP, TT, NT, VV>;
  constexpr int V = Gm::V, G = Gm::G, T = Gm::T;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  __syncthreads();   // the first DIF pass reads the top stages' twiddles
  const uint32_t item = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t tile = item % a.tiles;
  const uint64_t blk = item / a.tiles;
  const uint32_t lane0 = tile * T;
  ChirpLoad<V> ld{a.c + blk * a.st_c + lane0, a.ld_c, a.su, a.L, lane0, a.lanes, a.vec != 0};
  LdsLoad<V, G> ll{lds};
  LdsStore<V, G, false> sl{lds};
  LdsStore<V, G, true> slf{lds};
  ProductStore<V, G> prod{lds, a.vhat_br};
  ChirpStore<V> st{a.out + blk * a.st_o + lane0, a.ld_o, a.so, a.L, a.M, lane0, a.lanes, a.vec != 0};
  dif<LP, Gm::BM, V, G, false>(tws, ld, ll, slf, prod);
  dit<LP, Gm::BM, V, G, true>(tws, ll, ll, sl, st);
}

}  // namespace ct
}  // namespace fntrs
