// Transforms longer than a lane-wide tile (n = 2^14 .. 2^16): four-step FNT
// passes over 32-lane tiles.
//
// A transform of size N = N1*N2 (Sec. II-A, divide and conquer) is split as
//   X[m2 + N2 m1] = sum_i1 w_N1^(i1 m1) w_N^(i1 m2) sum_i2 x[i1 + N1 i2] w_N2^(i2 m2)
// pass A: for each i1, an N2-point transform over rows i1 + N1 i2, times the
//         twiddle w_N^(i1 m2), written to scratch row i1*N2 + m2;
// pass B: for each m2, an N1-point transform over scratch rows i1*N2 + m2,
//         giving outputs m2 + N2 m1.
// Each pass is an on-chip transform of one workgroup over a 32-lane tile
// (128-byte row segments), built on the compile-time passes of ctfnt.hpp.
// The decoder's three transforms (inverse FNT_n, FNT_M, inverse FNT_M) are
// chained so that pass B of one transform and pass A of the next share a
// workgroup: the output set {m2 + N2 m1 : m1} of pass B is exactly the input
// set of the next transform's pass A with N1' = N2.
#pragma once
#include "ct_kernels.hpp"
#include "fourstep_launch.hpp"

namespace fntrs {



namespace fs {

constexpr int kT = 32;       // lanes per tile
constexpr int kNT = 256;     // threads per workgroup
// Two lanes per thread: a 256-point pass then has an item for every thread
// (with four, half the threads would idle), and a ragged lane tail wastes
// less of a vector.
constexpr int kV = 2;

template <int L>
using Geo = ct::Geo<L, kT, kNT, kV>;

// scratch row stride: every scratch buffer is [block][row][lane], ld = lanes
// rounded up to the tile, rows = N.

// Decodes blockIdx into (lane tile, sub-transform, block).
struct Work {
  uint32_t tile, sub;
  uint64_t blk;
  uint32_t lane0;
};
__device__ __forceinline__ Work work_of(const FourStepArgs& a) {
  const uint32_t bid = ct::xcd_remap(blockIdx.x, gridDim.x);
  Work w;
  w.tile = bid % a.tiles;
  const uint32_t r = bid / a.tiles;
  w.sub = r % a.subs;
  w.blk = r / a.subs;
  w.lane0 = w.tile * kT;
  return w;
}

// Row r of a [block][row][lane] buffer, lane group g (V = 4 lanes).
__device__ __forceinline__ const uint32_t* rowp(const uint32_t* p, uint64_t ld, uint64_t r, uint32_t g) {
  return p + r * ld + g * kV;
}

template <int L, int V>
__device__ __forceinline__ void zero_item(int32_t (&x)[V]) {
#pragma unroll
  for (int v = 0; v < V; ++v) x[v] = 0;
}

// Generic global loader for the first DIT pass: position p of the size-2^L
// sub-transform holds input index i = bitrev(p); `row(i)` gives the row to
// read (or ~0u for a zero), `scale(i)` a per-row multiplier (0 = none).
// The reads of an item go out in three rounds -- the row descriptors (which
// may themselves be reads), then every row with no branch (a zero position
// reads row 0, which exists in every input, and is discarded), then the
// scaling -- so each round waits once for the whole item.
template <int L, class RowFn>
struct GLoad {
  const uint32_t* base;   // block base + lane0
  uint64_t ld;
  uint32_t lane0, lanes;
  bool vec;
  RowFn rowf;
  template <int B, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t ib, uint32_t g, int32_t (&x)[1 << B][kV]) {
    uint64_t r[1 << B];
    uint32_t w[1 << B];
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t i = ib | (bitrev((uint32_t)c, B) << (L - B));
      w[c] = 0;
      r[c] = rowf(i, w[c]);
    }
#pragma unroll
    for (int c = 0; c < (1 << B); ++c)
      ct::load_lanes<kV, WHOLE>(rowp(base, ld, r[c] == ~0ull ? 0 : r[c], g), lane0 + g * kV, lanes, x[c]);
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
#pragma unroll
      for (int v = 0; v < kV; ++v)
        x[c][v] = r[c] == ~0ull ? 0 : (w[c] ? (int32_t)ct::mulc((uint32_t)x[c][v], w[c]) : x[c][v]);
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t pb, uint32_t g, int32_t (&x)[1 << B][kV]) {
    static_assert(H == 1, "the first DIT pass has stride 1");
    const uint32_t ib = bitrev(pb, L);
    if (whole_vector<kV>(lane0 + g * kV, lanes, vec)) rows<B, true>(ib, g, x);
    else rows<B, false>(ib, g, x);
  }
};

// Generic global storer: position p holds output index m = p (natural, DIT)
// or m = bitrev(p) (DIF, REV); `dest(m, w)` gives the row (or ~0 to drop) and
// a multiplier w (0 = none) applied before the store.  The multipliers of an
// item (table reads) are all read before its first store: a read placed after
// a store could not be moved above it, and would wait on every row.
template <int L, bool REV, class DestFn>
struct GStore {
  uint32_t* base;
  uint64_t ld;
  uint32_t lane0, lanes;
  bool vec;
  DestFn destf;
  template <int B, uint32_t H, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t pb, uint32_t g, int32_t (&x)[1 << B][kV]) {
    uint64_t r[1 << B];
    uint32_t w[1 << B];
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t p = pb + c * H;
      w[c] = 0;
      r[c] = destf(REV ? bitrev(p, L) : p, w[c]);
    }
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      if (r[c] == ~0ull) continue;
      int32_t y[kV];
#pragma unroll
      for (int v = 0; v < kV; ++v) y[v] = w[c] ? ct::mulc(ct::canon(x[c][v]), w[c]) : x[c][v];
      ct::store_lanes<kV, WHOLE>(const_cast<uint32_t*>(rowp(base, ld, r[c], g)), lane0 + g * kV, lanes, y);
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t pb, uint32_t g, int32_t (&x)[1 << B][kV]) {
    if (whole_vector<kV>(lane0 + g * kV, lanes, vec)) rows<B, H, true>(pb, g, x);
    else rows<B, H, false>(pb, g, x);
  }
};

// Twiddle of the four-step split: w_N^(e) for a forward / inverse root of
// order N = 2^logN, e taken mod N.
__device__ __forceinline__ uint32_t tw4(const FourStepArgs& a, bool inv, uint32_t e, int logN) {
  const uint32_t idx = (e & ((1u << logN) - 1)) << (16 - logN);
  return inv ? gptr(a.twi)[idx] : gptr(a.tw)[idx];
}

// ------------------------------------------------------------------ kernels
// Decoder K1: inverse FNT_n pass A (N1 = n/256, N2 = 256).  Input index
// i2 -> position z = i1 + N1 i2 with weight wfull[z] (0 = erased).  Output
// Y[i1][m2] * w_n^-(i1 m2) to scratch row i1*256 + m2.
template <int LA>
__global__ void __launch_bounds__(kNT) k4_dec1(FourStepArgs a) {
  using Gm = Geo<LA>;
  extern __shared__ uint32_t lds[];
  const Work wk = work_of(a);
  const uint32_t i1 = wk.sub, N1 = a.n >> LA;
  auto rowf = [&](uint32_t i2, uint32_t& w) -> uint64_t {
    const uint32_t z = i1 + N1 * i2;
    w = gptr(a.wfull)[z];
    const uint32_t r = a.full ? z : gptr(a.ridx)[z];
    return w ? (uint64_t)r : ~0ull;
  };
  auto destf = [&](uint32_t m2, uint32_t& w) -> uint64_t {
    w = tw4(a, true, i1 * m2, a.logn);
    return (uint64_t)i1 * (1u << LA) + m2;
  };
  GLoad<LA, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.lane0, a.ld_in, wk.lane0, a.lanes, a.vec != 0, rowf};
  ct::LdsLoad<kV, Gm::G> lm{lds};
  ct::LdsStore<kV, Gm::G, false> sm{lds};
  GStore<LA, false, decltype(destf)> sl{a.out + wk.blk * a.stride_out + wk.lane0, a.ld_out, wk.lane0, a.lanes,
                                        a.vec != 0, destf};
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<LA, Gm::BM, kV, Gm::G, true>(tws, l0, lm, sm, sl);
}

// LDS storer that keeps index m only while index(m) < limit (else zero) and
// folds the values (a DIF transform follows).
template <int G>
struct MaskStore {
  uint32_t* lds;
  uint32_t m2, k;    // series index = m2 + 256 m
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t pb, uint32_t g, int32_t (&x)[1 << B][kV]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t m = pb + c * H;
#pragma unroll
      for (int v = 0; v < kV; ++v) x[c][v] = (m2 + 256u * m < k) ? ct::fold1(x[c][v]) : 0;
    }
    ct::lds_item_put<B, kV, G, H>(lds, pb, g, x);
  }
};

// Decoder K2: inverse FNT_n pass B (size N1 = 2^LB1 over scratch rows
// i1*256 + m2, m2 = sub) -> S at series indices m2 + 256 m1 (zero from k on)
// -> FNT_M pass A (size M/256 = 2^LB2, DIF, inputs m1 < M/256) -> times
// w_M^(m2 m2') -> scratch row m2*(M/256) + m2'.
template <int LB1, int LB2>
__global__ void __launch_bounds__(kNT) k4_dec2(FourStepArgs a) {
  using Gm = Geo<LB1>;
  extern __shared__ uint32_t lds[];
  const Work wk = work_of(a);
  const uint32_t m2 = wk.sub;
  auto rowf = [&](uint32_t i1, uint32_t& w) -> uint64_t {
    w = 0;
    return (uint64_t)i1 * 256u + m2;
  };
  auto destf = [&](uint32_t mp, uint32_t& w) -> uint64_t {
    w = tw4(a, false, m2 * mp, a.logm);
    return (uint64_t)m2 * (1u << LB2) + mp;
  };
  GLoad<LB1, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.lane0, a.ld_in, wk.lane0, a.lanes, a.vec != 0,
                                rowf};
  ct::LdsLoad<kV, Gm::G> ll{lds};
  ct::LdsStore<kV, Gm::G, false> sl{lds};
  ct::LdsStore<kV, Gm::G, true> slf{lds};
  MaskStore<Gm::G> ms{lds, m2, a.k};
  GStore<LB2, true, decltype(destf)> sg{a.out + wk.blk * a.stride_out + wk.lane0, a.ld_out, wk.lane0, a.lanes,
                                        a.vec != 0, destf};
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<LB1, Gm::BM, kV, Gm::G, true>(tws, l0, ll, sl, ms);
  ct::dif<LB2, Gm::BM, kV, Gm::G, false>(tws, ll, ll, slf, sg);
}

// LDS storer of the product: natural index m1' of FNT_M pass B with
// sub = m2' -> times ahat[m2' + (M/256) m1'] (which carries M^-1), folded.
template <int G>
struct AhatStore {
  uint32_t* lds;
  const uint32_t* ahat;
  uint32_t m2p, rows2;   // rows2 = M / 256
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t pb, uint32_t g, int32_t (&x)[1 << B][kV]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t h = gptr(ahat)[m2p + rows2 * (pb + c * H)];
#pragma unroll
      for (int v = 0; v < kV; ++v) x[c][v] = ct::mulc(ct::canon(x[c][v]), h);
    }
    ct::lds_item_put<B, kV, G, H>(lds, pb, g, x);
  }
};

// Decoder K3: FNT_M pass B (size 256 over scratch rows i1'*(M/256) + m2',
// m2' = sub) -> times Â -> inverse FNT_M pass A (size 256, DIF, N1'' = M/256
// so i1'' = m2') -> times w_M^-(m2' m2'') -> scratch row m2'*256 + m2''.
__global__ void __launch_bounds__(kNT) k4_dec3(FourStepArgs a) {
  using Gm = Geo<8>;
  extern __shared__ uint32_t lds[];
  const Work wk = work_of(a);
  const uint32_t m2p = wk.sub, rows2 = a.M >> 8;
  auto rowf = [&](uint32_t i1p, uint32_t& w) -> uint64_t {
    w = 0;
    return (uint64_t)i1p * rows2 + m2p;
  };
  auto destf = [&](uint32_t m2pp, uint32_t& w) -> uint64_t {
    w = tw4(a, true, m2p * m2pp, a.logm);
    return (uint64_t)m2p * 256u + m2pp;
  };
  GLoad<8, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.lane0, a.ld_in, wk.lane0, a.lanes, a.vec != 0, rowf};
  ct::LdsLoad<kV, Gm::G> ll{lds};
  ct::LdsStore<kV, Gm::G, false> sl{lds};
  ct::LdsStore<kV, Gm::G, true> slf{lds};
  AhatStore<Gm::G> ah{lds, a.ahat, m2p, rows2};
  GStore<8, true, decltype(destf)> sg{a.out + wk.blk * a.stride_out + wk.lane0, a.ld_out, wk.lane0, a.lanes,
                                      a.vec != 0, destf};
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<8, Gm::BM, kV, Gm::G, false>(tws, l0, ll, sl, ah);
  ct::dif<8, Gm::BM, kV, Gm::G, true>(tws, ll, ll, slf, sg);
}

// Decoder K4 / last pass of an inverse transform: size 2^LB over scratch rows
// i1*256 + m2 (m2 = sub) -> outputs m2 + 256 m1 < k to the destination.
template <int LB>
__global__ void __launch_bounds__(kNT) k4_dec4(FourStepArgs a) {
  using Gm = Geo<LB>;
  extern __shared__ uint32_t lds[];
  const Work wk = work_of(a);
  const uint32_t m2 = wk.sub;
  auto rowf = [&](uint32_t i1, uint32_t& w) -> uint64_t {
    w = 0;
    return (uint64_t)i1 * 256u + m2;
  };
  auto destf = [&](uint32_t m1, uint32_t& w) -> uint64_t {
    w = 0;
    const uint32_t m = m2 + 256u * m1;
    return m < a.k ? (uint64_t)m : ~0ull;
  };
  GLoad<LB, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.lane0, a.ld_in, wk.lane0, a.lanes, a.vec != 0,
                               rowf};
  ct::LdsLoad<kV, Gm::G> ll{lds};
  ct::LdsStore<kV, Gm::G, false> sl{lds};
  GStore<LB, false, decltype(destf)> sg{a.out + wk.blk * a.stride_out + wk.lane0, a.ld_out, wk.lane0, a.lanes,
                                        a.vec != 0, destf};
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<LB, Gm::BM, kV, Gm::G, true>(tws, l0, ll, sl, sg);
}

// Encoder as one FNT_n of the zero-padded source, n = N1 * 256.  Pass A:
// rows i1 + N1 i2 (zero from k on), forward, times w_n^(i1 m2) -> scratch
// row i1*256 + m2.
__global__ void __launch_bounds__(kNT) k4_enc1(FourStepArgs a) {
  using Gm = Geo<8>;
  extern __shared__ uint32_t lds[];
  const Work wk = work_of(a);
  const uint32_t i1 = wk.sub, N1 = a.n >> 8;
  auto rowf = [&](uint32_t i2, uint32_t& w) -> uint64_t {
    w = 0;
    const uint32_t j = i1 + N1 * i2;
    return j < a.k ? (uint64_t)j : ~0ull;
  };
  auto destf = [&](uint32_t m2, uint32_t& w) -> uint64_t {
    w = tw4(a, false, i1 * m2, a.logn);
    return (uint64_t)i1 * 256u + m2;
  };
  GLoad<8, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.lane0, a.ld_in, wk.lane0, a.lanes, a.vec != 0, rowf};
  ct::LdsLoad<kV, Gm::G> lm{lds};
  ct::LdsStore<kV, Gm::G, false> sm{lds};
  GStore<8, false, decltype(destf)> sl{a.out + wk.blk * a.stride_out + wk.lane0, a.ld_out, wk.lane0, a.lanes,
                                       a.vec != 0, destf};
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<8, Gm::BM, kV, Gm::G, false>(tws, l0, lm, sm, sl);
}

// Encoder pass B (size N1 = 2^LB): scratch rows i1*256 + m2 (m2 = sub),
// forward -> rows m2 + 256 m1.
template <int LB>
__global__ void __launch_bounds__(kNT) k4_enc2(FourStepArgs a) {
  using Gm = Geo<LB>;
  extern __shared__ uint32_t lds[];
  const Work wk = work_of(a);
  const uint32_t m2 = wk.sub;
  auto rowf = [&](uint32_t i1, uint32_t& w) -> uint64_t {
    w = 0;
    return (uint64_t)i1 * 256u + m2;
  };
  auto destf = [&](uint32_t m1, uint32_t& w) -> uint64_t {
    w = 0;
    const uint32_t r = m2 + 256u * m1;
    return (a.rows_out && r >= a.rows_out) ? ~0ull : (uint64_t)r;
  };
  GLoad<LB, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.lane0, a.ld_in, wk.lane0, a.lanes, a.vec != 0, rowf};
  ct::LdsLoad<kV, Gm::G> lm{lds};
  ct::LdsStore<kV, Gm::G, false> sm{lds};
  GStore<LB, false, decltype(destf)> sl{a.out + wk.blk * a.stride_out + wk.lane0, a.ld_out, wk.lane0, a.lanes,
                                       a.vec != 0, destf};
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<LB, Gm::BM, kV, Gm::G, false>(tws, l0, lm, sm, sl);
}

}  // namespace fs
}  // namespace fntrs
