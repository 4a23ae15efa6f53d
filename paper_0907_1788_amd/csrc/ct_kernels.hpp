// Encoder and decoder kernels on compile-time transform plans (ctfnt.hpp).
// One workgroup owns a tile of T lanes of one codeword block; every
// transform of that block runs on chip, so each block crosses HBM once in
// each direction.
#pragma once
#include "codec_args.hpp"
#include "ctfnt.hpp"

#include <type_traits>

namespace fntrs {
namespace ct {

// Radix bound of the pass plan for a size-2^L transform on G lane groups of V
// lanes: aim for kThreads items per pass (items = G 2^(L-B)), radix 8 at
// least, the register budget of V lanes at most, and no more passes than
// needed while a pass keeps at least half the threads busy.
__host__ __device__ constexpr int geo_bm(int L, int G, int V, int NT) {
  int lg = 0, lt = 0;
  while ((1 << lg) < G) ++lg;
  while ((1 << lt) < NT) ++lt;
  // radix 2^5 at most: a first pass of trivial butterflies grows a value by
  // 2^B and the multiplier takes 24-bit operands
  const int bmax = V == 4 ? 4 : 5;
  int b = L + lg - lt;
  if (b < 3) b = 3;
  if (b > bmax) b = bmax;
  if (b > L) b = L;
  if (b < 1) b = 1;
  // a larger radix that saves a pass while items >= kThreads/2
  for (int c = b + 1; c <= bmax && c <= L; ++c)
    if ((L + c - 1) / c < (L + b - 1) / b && (G << (L - c)) >= NT / 2) return c;
  return b;
}

// Tile geometry: T lanes per tile, V lanes per thread (VV, or 4 when the
// tile allows), G = T/V lane groups, NT threads, radix bound BM, LDS bytes of
// the padded tile.
template <int L, int T_, int NT_, int VV = 0>
struct Geo {
  static constexpr int T = T_;
  static constexpr int NT = NT_;
  static constexpr int V = VV ? VV : (T >= 4 ? 4 : T);   // lanes per thread (vector width)
  static_assert(T % V == 0, "the tile must hold whole vectors");
  static constexpr int G = T / V;
  static constexpr int BM = geo_bm(L, G, V, NT);
  static constexpr uint32_t TILE_BYTES = lds_vectors(1u << L, G) * V * 4;
  // LDS twiddle tables (TwLds): stages from the second pass up; all stages in
  // per-stage tables when they fit, else the top two stages share the
  // stage-L table; none when even that does not fit (global tables then)
  // (the decoder's size-2^(L-1) transforms start with their own first pass)
  static constexpr int LO = (L > 1 && plan_b(L - 1, BM, 0) < plan_b(L, BM, 0) ? plan_b(L - 1, BM, 0)
                                                                                : plan_b(L, BM, 0)) + 1;
  static constexpr uint32_t WORDS_ALL = TwLds<L, LO, L>::words();
  static constexpr uint32_t WORDS_TOP2 = TwLds<L, LO, L - 2>::words();
  static constexpr int TOP = TILE_BYTES + WORDS_ALL * 4 <= 163840 ? L : L - 2;
  static constexpr bool TW_LDS = TILE_BYTES + (TOP == L ? WORDS_ALL : WORDS_TOP2) * 4 <= 163840 && LO <= L;
  static constexpr uint32_t LDS_BYTES = TILE_BYTES + (TW_LDS ? (TOP == L ? WORDS_ALL : WORDS_TOP2) * 4 : 0);
  using TwType = typename std::conditional<TW_LDS, TwLds<L, LO, TOP>, TwGlobal>::type;
};

template <int L, int LO, int TOP>
__device__ __forceinline__ TwLds<L, LO, TOP> make_tw(const TwLds<L, LO, TOP>*, uint32_t* lds_tab, const uint32_t* tw,
                                                      const uint32_t*) {
  TwLds<L, LO, TOP> t{lds_tab};
  t.fill(lds_tab, tw);
  return t;
}
__device__ __forceinline__ TwGlobal make_tw(const TwGlobal*, uint32_t*, const uint32_t* tw, const uint32_t* twi) {
  return TwGlobal{tw, twi};
}

// ---------------------------------------------------------------- LDS movers
template <int V, int G>
struct LdsLoad {
  const uint32_t* lds;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    lds_item_get<B, V, G, H>(lds, base, g, x);
  }
};

template <int V, int G, bool FOLD>
struct LdsStore {
  uint32_t* lds;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    if constexpr (FOLD) {
#pragma unroll
      for (int c = 0; c < (1 << B); ++c)
#pragma unroll
        for (int v = 0; v < V; ++v) x[c][v] = fold1(x[c][v]);
    }
    lds_item_put<B, V, G, H>(lds, base, g, x);
  }
};

// 64-bit row address helper: rows are `ld` elements apart.
__device__ __forceinline__ const uint32_t* row_ptr(const uint32_t* p, uint64_t row, uint64_t ld) {
  return p + row * ld;
}

template <int V>
__device__ __forceinline__ void load_lanes(const uint32_t* p, uint32_t lane, uint32_t lanes, bool vec,
                                           int32_t (&x)[V]) {
  uint32_t u[V];
  gload<V>(p, lane, lanes, vec, u);
#pragma unroll
  for (int v = 0; v < V; ++v) x[v] = (int32_t)u[v];
}

template <int V>
__device__ __forceinline__ void store_lanes(uint32_t* p, uint32_t lane, uint32_t lanes, bool vec,
                                            const int32_t (&x)[V]) {
  uint32_t u[V];
#pragma unroll
  for (int v = 0; v < V; ++v) u[v] = canon(x[v]);
  gstore<V>(p, lane, lanes, vec, u);
}

// ---------------------------------------------------------------- encoder
// First DIT pass of the encoder: position pos holds source row bitrev(pos),
// twisted by r_n^(t j) (coset t); rows j >= k are zero padding.
template <int L, int V>
struct EncLoad {
  const uint32_t* src;
  const uint32_t* tw;
  uint64_t ld;
  uint32_t k, n, t, lane0, lanes;
  int sh;
  bool vec;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    static_assert(H == 1, "the first DIT pass has stride 1");
    const uint32_t jb = bitrev(base, L);
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t j = jb | (bitrev((uint32_t)c, B) << (L - B));
      if (j < k) {
        load_lanes<V>(row_ptr(src, j, ld) + g * V, lane0 + g * V, lanes, vec, x[c]);
        if (t) {
          const uint32_t w = tw[((t * j) & (n - 1)) << sh];
#pragma unroll
          for (int v = 0; v < V; ++v) x[c][v] = mulw(x[c][v], w);
        }
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) x[c][v] = 0;
      }
    }
  }
};

// Last DIT pass of the encoder: output m of coset t is row t + cosets*m.
template <int V>
struct EncStore {
  uint32_t* dst;
  uint64_t ld;
  uint32_t t, cosets, lane0, lanes;
  bool vec;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint64_t row = t + (uint64_t)cosets * (base + c * H);
      store_lanes<V>(dst + row * ld + g * V, lane0 + g * V, lanes, vec, x[c]);
    }
  }
};

// Encoder, Sec. II-B: e_i = s(r_n^i).  Output row t + (n/K) m is output m of
// FNT_K of (s_j r_n^(t j))_j (r_n^(n/K) = r_K), one work item per
// (coset t, lane tile, block), coset fastest.
template <int LK, int TT, int NT, int VV, class TW>
__device__ __forceinline__ void enc_item(const EncodeArgs& a, uint32_t item, uint32_t* lds, const TW& tws) {
  using Gm = Geo<LK, TT, NT, VV>;
  constexpr int V = Gm::V, G = Gm::G, T = Gm::T;
  const uint32_t t = item % a.cosets;
  item /= a.cosets;
  const uint32_t tile = item % a.tiles;
  const uint64_t blk = item / a.tiles;
  const uint32_t lane0 = tile * T;
  EncLoad<LK, V> l0{a.src + blk * a.stride_src + lane0, a.tw, a.ld_src, a.k, a.n, t, lane0, a.lanes,
                    16 - a.logn, a.vec != 0};
  LdsLoad<V, G> lm{lds};
  LdsStore<V, G, false> sm{lds};
  EncStore<V> sl{a.dst + blk * a.stride_dst + lane0, a.ld_dst, t, a.cosets, lane0, a.lanes, a.vec != 0};
  dit<LK, Gm::BM, V, G, false>(tws, l0, lm, sm, sl);
}

template <int LK, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_enc(EncodeArgs a) {
  using Gm = Geo<LK, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  enc_item<LK, TT, NT, VV>(a, xcd_remap(blockIdx.x, gridDim.x), lds, tws);
}

// Job of work item w: the last j with start[j] <= w (uniform per workgroup).
__device__ __forceinline__ uint32_t find_job(const uint32_t* start, uint32_t njobs, uint32_t w) {
  uint32_t lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (start[mid] <= w) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Batched encoder: a persistent grid walks the work items of every job of
// one transform size; the LDS twiddle tables are filled once per workgroup.
template <int LK, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_enc_tab(JobTable<EncodeArgs> t, const uint32_t* tw, const uint32_t* twi) {
  using Gm = Geo<LK, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, tw, twi);
  for (uint32_t w = xcd_remap(blockIdx.x, gridDim.x); w < t.total; w += gridDim.x) {
    const uint32_t j = find_job(t.start, t.njobs, w);
    const EncodeArgs a = t.jobs[j];
    enc_item<LK, TT, NT, VV>(a, w - t.start[j], lds, tws);
    __syncthreads();   // the next item overwrites the LDS tile
  }
}

// ---------------------------------------------------------------- decoder
// First DIT pass of step 5: position pos holds u at index z = bitrev(pos):
// the received symbol v_z times the locator weight of z (0 if z is erased).
template <int L, int V>
struct DecLoad {
  const uint32_t* recv;
  const uint32_t* wfull;
  const uint32_t* ridx;
  uint64_t ld;
  uint32_t lane0, lanes;
  bool full, vec;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    static_assert(H == 1, "the first DIT pass has stride 1");
    const uint32_t zb = bitrev(base, L);
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t z = zb | (bitrev((uint32_t)c, B) << (L - B));
      const uint32_t w = wfull[z];
      if (w) {
        const uint32_t row = full ? z : ridx[z];
        load_lanes<V>(row_ptr(recv, row, ld) + g * V, lane0 + g * V, lanes, vec, x[c]);
#pragma unroll
        for (int v = 0; v < V; ++v) x[c][v] = mulc((uint32_t)x[c][v], w);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) x[c][v] = 0;
      }
    }
  }
};

// Last pass of step 5: keep S_m = U_m for m < k (folded: the DIF transform
// that follows doubles ranges), zero for k <= m < M (the padding of the
// length-M product), positions >= M are never read.
template <int V, int G>
struct SeriesStore {
  uint32_t* lds;
  uint32_t k;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t m = base + c * H;
#pragma unroll
      for (int v = 0; v < V; ++v) x[c][v] = m < k ? fold1(x[c][v]) : 0;
    }
    // positions >= 2k are never read again; writing them is harmless
    lds_item_put<B, V, G, H>(lds, base, g, x);
  }
};

// Last DIF pass of step 6: multiply the transform of S (bit-reversed order)
// by the locator's FNT_2k(A mod x^k)/2k, stored in the same order.
template <int V, int G>
struct ProductStore {
  uint32_t* lds;
  const uint32_t* ahat_br;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t h = ahat_br[base + c * H];
#pragma unroll
      for (int v = 0; v < V; ++v) x[c][v] = mulc(canon(x[c][v]), h);
    }
    lds_item_put<B, V, G, H>(lds, base, g, x);
  }
};

// Last DIT pass of step 6: coefficients m < k are the recovered source rows.
template <int V>
struct SourceStore {
  uint32_t* dst;
  uint64_t ld;
  uint32_t k, lane0, lanes;
  bool vec;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t m = base + c * H;
      if (m < k) store_lanes<V>(dst + (uint64_t)m * ld + g * V, lane0 + g * V, lanes, vec, x[c]);
    }
  }
};

// Decoder, Sec. II-B steps 4-6, for n = 2^LN, k < n, and a product length
// M = 2^(LN-D) >= 2k (D in {0, 1}; any cyclic length >= 2k-1 makes the
// low product exact):
//   step 4+5: u_z = weight_z v_z (the locator folds -x_z^(-1)/A'(x_z) into
//             the weight), S_j = sum_z u_z r^(-j z) for j < k: inverse DIT
//             FNT_n, inputs read from global memory in bit-reversed order;
//   step 6:   P = (A S) mod x^k: DIF FNT_M of (S, 0) (natural in,
//             bit-reversed out), times FNT_M(A mod x^k)/M, inverse DIT FNT_M
//             (bit-reversed in, natural out); keep m < k.
// No permutation passes through LDS between the three transforms.
// D = -1 is the erasure-free case k = n (Sec. II-B): the weights are n^-1
// and the inverse FNT_n alone is the decoder.
template <int LN, int D, int TT, int NT, int VV, class TW>
__device__ __forceinline__ void dec_item(const DecodeArgs& a, uint32_t item, uint32_t* lds, const TW& tws) {
  using Gm = Geo<LN, TT, NT, VV>;
  constexpr int V = Gm::V, G = Gm::G, T = Gm::T;
  const uint32_t tile = item % a.tiles;
  const uint64_t blk = item / a.tiles;
  const uint32_t lane0 = tile * T;
  DecLoad<LN, V> lg{a.recv + blk * a.stride_recv + lane0, a.wfull, a.ridx, a.ld_recv, lane0, a.lanes,
                    a.full != 0, a.vec != 0};
  LdsLoad<V, G> ll{lds};
  LdsStore<V, G, false> sl{lds};
  SourceStore<V> sg{a.dst + blk * a.stride_dst + lane0, a.ld_dst, a.k, lane0, a.lanes, a.vec != 0};
  if constexpr (D < 0) {
    dit<LN, Gm::BM, V, G, true>(tws, lg, ll, sl, sg);
  } else {
    constexpr int L2 = LN - D;
    LdsStore<V, G, true> slf{lds};
    SeriesStore<V, G> ss{lds, a.k};
    ProductStore<V, G> sp{lds, a.ahat_br};
    dit<LN, Gm::BM, V, G, true>(tws, lg, ll, sl, ss);
    dif<L2, Gm::BM, V, G, false>(tws, ll, ll, slf, sp);
    dit<L2, Gm::BM, V, G, true>(tws, ll, ll, sl, sg);
  }
}

template <int LN, int D, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_dec(DecodeArgs a) {
  using Gm = Geo<LN, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  dec_item<LN, D, TT, NT, VV>(a, xcd_remap(blockIdx.x, gridDim.x), lds, tws);
}

// Batched decoder: as k_enc_tab, for decode jobs of one code length n and
// one product length M = n / 2^D, each with its own locator.
template <int LN, int D, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_dec_tab(JobTable<DecodeArgs> t, const uint32_t* tw, const uint32_t* twi) {
  using Gm = Geo<LN, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, tw, twi);
  for (uint32_t w = xcd_remap(blockIdx.x, gridDim.x); w < t.total; w += gridDim.x) {
    const uint32_t j = find_job(t.start, t.njobs, w);
    const DecodeArgs a = t.jobs[j];
    dec_item<LN, D, TT, NT, VV>(a, w - t.start[j], lds, tws);
    __syncthreads();
  }
}

}  // namespace ct
}  // namespace fntrs
