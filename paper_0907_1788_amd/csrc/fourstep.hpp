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

constexpr int kT = kFourStepTile;   // lanes per tile
#ifndef FNTRS_FS_THREADS
#define FNTRS_FS_THREADS 256
#endif
#ifndef FNTRS_FS_V
#define FNTRS_FS_V 2
#endif
constexpr int kNT = FNTRS_FS_THREADS;   // threads per workgroup
// Two lanes per thread: a 256-point pass then has an item for every thread
// (with four, half the threads would idle), and a ragged lane tail wastes
// less of a vector.
constexpr int kV = FNTRS_FS_V;

template <int L>
using Geo = ct::Geo<L, kT, kNT, kV>;

// Buffers are addressed per lane tile: element (block b, row r, lane
// tile*kT + l) lies at b*stride + tile*tstride + r*ld + l.  Input and output
// buffers are row-major (tstride = kT, ld = lanes); scratch is tile-major
// ([block][tile][row][kT]: tstride = rows*kT, ld = kT), so a workgroup's
// rows of one tile lie in one contiguous region of rows*128 bytes instead of
// being spread over the whole buffer at a stride of ld*4 bytes.

// Decodes blockIdx into (lane tile, sub-transform, block).  Consecutive
// work items of one XCD run together and share its L2, so the order decides
// which workgroups share cache lines while they are in flight:
//   0  lane tile first: neighbouring tiles share the lines of a row-major
//      buffer whose lane count is not a multiple of the tile;
//   1  sub-transform first: neighbouring sub-transforms share the 128-byte
//      lines of the scratch rows they read (two 64-byte rows of one tile);
//   2  pairs of sub-transforms, then tiles: both, for kernels that read
//      scratch and write row-major rows.
struct Work {
  uint32_t tile, sub;
  uint64_t blk;
  uint32_t lane0;
};
__device__ __forceinline__ Work work_of(const FourStepArgs& a) {
  const uint32_t bid = ct::xcd_remap(blockIdx.x, gridDim.x);
  Work w;
  if (a.order == 1) {
    w.sub = bid % a.subs;
    const uint32_t r = bid / a.subs;
    w.tile = r % a.tiles;
    w.blk = r / a.tiles;
  } else if (a.order == 2) {   // subs is even
    const uint32_t rest = bid >> 1, half = a.subs >> 1;
    w.tile = rest % a.tiles;
    const uint32_t r = rest / a.tiles;
    w.sub = ((r % half) << 1) | (bid & 1u);
    w.blk = r / half;
  } else {
    w.tile = bid % a.tiles;
    const uint32_t r = bid / a.tiles;
    w.sub = r % a.subs;
    w.blk = r / a.subs;
  }
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

// Scratch rows move as whole vectors of kV lanes: every lane tile of a
// scratch buffer is complete (the first kernel writes its padding lanes,
// which it reads as zero) and vectors are kV-aligned.  They hold canonical
// residues in 17 bits: the low 16 bits of a thread's two lanes share one
// word at element index e (byte 2e of the buffer).  Bit 16 is set only for
// 65536, about once in 2^16 elements, so it is stored by exception: where a
// lane of a row of a tile holds 65536, the row's 16 threads store one byte
// each at foff + e/2 (bit 0: first lane, bit 1: second) and the row's bit is
// set in an escape bitmap at boff.  That bitmap is cleared before the writer
// runs and ordered by reader: a writer's rows are i*S + m and row i*S + m is
// bit m*(R/S) + i of its tile's R bits, so the R/S rows one reading
// sub-transform m takes are R/S consecutive bits.  A reader whose bits are
// all clear (most of them) reads no flag byte.
static_assert(kV == 2, "scratch packs the two lanes of a thread");
__device__ __forceinline__ void scratch_get(const uint32_t* org, const uint32_t* p, int32_t (&x)[kV]) {
  const uint64_t e = (uint64_t)(p - org);
  const uint32_t t = *(const FNTRS_GLOBAL uint32_t*)gptr((const uint32_t*)((const uint16_t*)org + e));
  x[0] = (int32_t)(t & 0xFFFFu);
  x[1] = (int32_t)(t >> 16);
}
__device__ __forceinline__ void scratch_fix(const uint32_t* org, uint64_t foff, const uint32_t* p, int32_t (&x)[kV]) {
  const uint64_t e = (uint64_t)(p - org);
  const uint32_t f = *(const FNTRS_GLOBAL uint8_t*)gptr((const uint8_t*)org + foff + (e >> 1));
  x[0] |= (int32_t)((f & 1u) << 16);
  x[1] |= (int32_t)((f & 2u) << 15);
}
// y: lazy values (|y| < 2^23), stored canonical; bit: the row's bit in the
// escape bitmap (uint32 words at bmap).  Called by all 16 threads of a row
// (lanes 16j .. 16j+15 of a wave) together.
__device__ __forceinline__ void scratch_put(const uint32_t* org, uint64_t foff, uint32_t* bmap, uint64_t bit,
                                            uint32_t* p, const int32_t (&y)[kV]) {
  const uint64_t e = (uint64_t)(p - org);
  const uint32_t c0 = ct::canon(y[0]), c1 = ct::canon(y[1]);
  *(FNTRS_GLOBAL uint32_t*)gptr((uint32_t*)((uint16_t*)org + e)) = (c0 & 0xFFFFu) | (c1 << 16);
  const uint32_t f = (c0 >> 16) | ((c1 >> 16) << 1);
  const uint64_t any = __ballot(f != 0);
  if ((any >> (threadIdx.x & 48u)) & 0xFFFFu) {
    *(FNTRS_GLOBAL uint8_t*)gptr((uint8_t*)org + foff + (e >> 1)) = (uint8_t)f;
    if ((threadIdx.x & 15u) == 0) atomicOr(bmap + (bit >> 5), 1u << (bit & 31u));
  }
}

// Where a loader's rows come from and what it does to them:
//   kScratch  - a tile-major scratch buffer (row stride kT), values as read;
//   kZeros    - the caller's input; rows the row function maps to ~0 are zero
//               and not read;
//   kWeighted - the caller's input times a per-row weight (0: the row is
//               erased and reads as zero; the row function then names any
//               existing row).
enum LoadKind { kScratch = 0, kZeros = 1, kWeighted = 2 };

// Global loader for the first DIT pass: position p of the size-2^L
// sub-transform holds input index i = bitrev(p); `row(i, w)` gives the row to
// read and (kWeighted) its weight.  The reads of an item go out in three
// rounds -- the row descriptors (which may themselves be reads), then the
// rows, then the weights -- so each round waits once for the
// whole item (zero rows of kZeros excepted).
// REP > 0 (kZeros): every input index i >= 2^(L-REP) is a zero row, i.e.
// every position p with a nonzero low REP bits.  The first REP DIT stages
// then only copy: each group of 2^REP positions ends up holding its first
// value (the lower element of every pair is zero before its stage).  The
// loader makes those copies and the pass starts at stage REP (kSkip).
template <int L, int KIND, class RowFn, int REP = 0>
struct GLoad {
  static_assert(REP == 0 || KIND == kZeros, "only zero rows can be skipped");
  static constexpr int kSkip = REP;
  const uint32_t* base;   // block base + lane tile
  uint64_t ld;
  uint32_t lane0, lanes;
  bool vec;
  RowFn rowf;
  const uint32_t* org = nullptr;   // kScratch: the buffer's origin and the
  uint64_t foff = 0;               // byte offset of its flags
  // kScratch: whether a row of this sub-transform holds 65536, and the word
  // of the escape bitmap where its 2^L bits start
  bool esc = false;
  const uint32_t* bm = nullptr;
  uint64_t w0 = 0;
  // Reads the escape bits of sub-transform `sub` of tile (blk, tile) of a
  // buffer of 2^rlog rows per tile.  Uniform, before any store of the kernel.
  __device__ __forceinline__ void escapes(const FourStepArgs& a, const Work& wk) {
    static_assert(L >= 5, "a sub-transform's escape bits are whole words");
    bm = (const uint32_t*)((const uint8_t*)org + a.boff_in);
    w0 = (((wk.blk * a.tiles + wk.tile) << a.rlog_in) + ((uint64_t)wk.sub << L)) >> 5;
    uint32_t any = 0;
#pragma unroll
    for (int j = 0; j < (1 << (L - 5)); ++j) any |= gptr(bm)[w0 + j];
    esc = any != 0;
  }
  template <int B, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t ib, uint32_t g, int32_t (&x)[1 << B][kV]) {
    uint64_t r[1 << B];
    uint32_t w[1 << B];
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t i = ib | (bitrev((uint32_t)c, B) << (L - B));
      w[c] = 1;
      r[c] = rowf(i, w[c]);
    }
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      if constexpr (KIND == kScratch) {
        scratch_get(org, base + r[c] * kT + g * kV, x[c]);
      } else if constexpr (KIND == kZeros) {
        // zero rows (the encoder's padding: the top rows of every
        // sub-transform, a whole wave at a time) issue no read
        if (r[c] != ~0ull) ct::load_lanes<kV, WHOLE>(rowp(base, ld, r[c], g), lane0 + g * kV, lanes, x[c]);
        else
#pragma unroll
          for (int v = 0; v < kV; ++v) x[c][v] = 0;
      } else {
        ct::load_lanes<kV, WHOLE>(rowp(base, ld, r[c], g), lane0 + g * kV, lanes, x[c]);
      }
    }
    if constexpr (KIND == kScratch) {
      if (esc) {   // uniform: a row of this sub-transform holds 65536
#pragma unroll
        for (int c = 0; c < (1 << B); ++c) {
          const uint32_t i = ib | (bitrev((uint32_t)c, B) << (L - B));
          if ((gptr(bm)[w0 + (i >> 5)] >> (i & 31u)) & 1u) {
            uint32_t unused;   // the row again: r[] need not live past the loads
            scratch_fix(org, foff, base + rowf(i, unused) * kT + g * kV, x[c]);
          }
        }
      }
    }
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
#pragma unroll
      for (int v = 0; v < kV; ++v)
        if constexpr (KIND == kWeighted) x[c][v] = ct::mulw(x[c][v], w[c]);
    }
    if constexpr (REP > 0) {
      static_assert(REP <= B, "the first pass covers the copied stages");
      constexpr int mask = (1 << REP) - 1;
#pragma unroll
      for (int c = 0; c < (1 << B); ++c)
        if (c & mask)
#pragma unroll
          for (int v = 0; v < kV; ++v) x[c][v] = x[c & ~mask][v];
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t pb, uint32_t g, int32_t (&x)[1 << B][kV]) {
    static_assert(H == 1, "the first DIT pass has stride 1");
    const uint32_t ib = bitrev(pb, L);
    if (KIND == kScratch || whole_vector<kV>(lane0 + g * kV, lanes, vec)) rows<B, true>(ib, g, x);
    else rows<B, false>(ib, g, x);
  }
};

// Global storer: position p holds output index m = p (natural, DIT) or
// m = bitrev(p) (DIF, REV); `dest(m, w)` gives the row and, for a scratch
// destination, the twiddle w it is multiplied by (lazy result) before the
// store; for the caller's output it gives the row or ~0 (drop), and values
// are stored canonical.  The twiddles of an item (table reads) are all read
// before its first store: a read placed after a store could not be moved
// above it, and would wait on every row.
template <int L, bool REV, bool SCRATCH, class DestFn>
struct GStore {
  uint32_t* base;
  uint64_t ld;
  uint32_t lane0, lanes;
  bool vec;
  DestFn destf;
  const uint32_t* org = nullptr;   // SCRATCH: the buffer's origin and the
  uint64_t foff = 0;               // byte offset of its flags
  uint32_t* bmap = nullptr;        // SCRATCH: escape bitmap words
  uint64_t bbit = 0;               // first bit of this tile
  uint32_t slog = 0, qlog = 0;     // log2 S and log2 R/S
  __device__ __forceinline__ void escapes(const FourStepArgs& a, const Work& wk) {
    bmap = (uint32_t*)((uint8_t*)a.out + a.boff_out);
    bbit = (wk.blk * a.tiles + wk.tile) << a.rlog_out;
    slog = a.slog_out;
    qlog = a.rlog_out - a.slog_out;
  }
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
      if constexpr (SCRATCH) {
        int32_t y[kV];
#pragma unroll
        for (int v = 0; v < kV; ++v) y[v] = ct::mulw(x[c][v], w[c]);
        const uint64_t bit = bbit + ((r[c] & ((1u << slog) - 1)) << qlog) + (r[c] >> slog);
        scratch_put(org, foff, bmap, bit, base + r[c] * kT + g * kV, y);
      } else {
        if (r[c] == ~0ull) continue;
        ct::store_lanes<kV, WHOLE>(const_cast<uint32_t*>(rowp(base, ld, r[c], g)), lane0 + g * kV, lanes, x[c]);
      }
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t pb, uint32_t g, int32_t (&x)[1 << B][kV]) {
    if (SCRATCH || whole_vector<kV>(lane0 + g * kV, lanes, vec)) rows<B, H, true>(pb, g, x);
    else rows<B, H, false>(pb, g, x);
  }
};

// Per-workgroup tables of the per-row factors of a tile (decoder weights and
// rows, split twiddles, the locator's transform): each word is read from
// global memory once per workgroup, one word per thread, into LDS behind the
// tile, instead of by every lane group at every row of its items -- those
// broadcast reads would otherwise keep the vector memory pipeline busy.
constexpr uint32_t kTabWords = 3 * 256;
template <int L>
constexpr uint32_t lds_with_tables() { return Geo<L>::LDS_BYTES + kTabWords * 4; }

// ------------------------------------------------------------------ kernels
// Decoder K1: inverse FNT_n pass A (N1 = n/256, N2 = 256).  Input index
// i2 -> position z = i1 + N1 i2 with weight wfull[z] (0 = erased).  Output
// Y[i1][m2] * w_n^-(i1 m2) to scratch row i1*256 + m2.
template <int LA>
__global__ void __launch_bounds__(kNT) k4_dec1(FourStepArgs a) {
  using Gm = Geo<LA>;
  extern __shared__ uint32_t lds[];
  const Work wk = work_of(a);
  const uint32_t i1 = wk.sub;
  // the weights, rows and last-pass twiddles of the 256 inputs go to LDS
  // tables first, one word per thread, so the first pass's lane groups do
  // not each read them again from global memory
  uint32_t* t_tw = lds + Gm::LDS_BYTES / 4;   // w_n^-(i1 m2)
  static_assert((3u << LA) <= kTabWords, "three tables of 2^LA words");
  uint32_t* t_w = t_tw + (1u << LA);           // weight of input i2
  uint32_t* t_r = t_w + (1u << LA);            // its row (0 where erased)
  for (uint32_t t = threadIdx.x; t < (1u << LA); t += kNT) {
    const u32x2 wr = *(const FNTRS_GLOBAL u32x2*)gptr(a.wr + 2 * (((uint64_t)i1 << LA) + t));
    t_tw[t] = gptr(a.twsplit)[((uint64_t)i1 << LA) + t];
    t_w[t] = wr.x;
    t_r[t] = wr.y;
  }
  __syncthreads();
  auto rowf = [&](uint32_t i2, uint32_t& w) -> uint64_t {
    w = t_w[i2];   // 0: erased (the row read is then discarded)
    return (uint64_t)t_r[i2];
  };
  auto destf = [&](uint32_t m2, uint32_t& w) -> uint64_t {
    w = t_tw[m2];
    return (uint64_t)i1 * (1u << LA) + m2;
  };
  GLoad<LA, kWeighted, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.tile * a.tstride_in, a.ld_in, wk.lane0,
                                          a.lanes, a.vec != 0, rowf};
  ct::LdsLoad<kV, Gm::G> lm{lds};
  ct::LdsStore<kV, Gm::G, false> sm{lds};
  GStore<LA, false, true, decltype(destf)> sl{a.out + wk.blk * a.stride_out + wk.tile * a.tstride_out, a.ld_out, wk.lane0, a.lanes,
                                        a.vec != 0, destf, a.out, a.foff_out};
  sl.escapes(a, wk);
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
  uint32_t* t_tw = lds + Gm::LDS_BYTES / 4;   // w_M^(m2 mp), read after the first barrier
  for (uint32_t t = threadIdx.x; t < (1u << LB2); t += kNT) t_tw[t] = gptr(a.twsplit)[(m2 << LB2) + t];
  auto rowf = [&](uint32_t i1, uint32_t& w) -> uint64_t {
    w = 0;
    return (uint64_t)i1 * 256u + m2;
  };
  auto destf = [&](uint32_t mp, uint32_t& w) -> uint64_t {
    w = t_tw[mp];
    return (uint64_t)m2 * (1u << LB2) + mp;
  };
  GLoad<LB1, kScratch, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.tile * a.tstride_in, a.ld_in, wk.lane0, a.lanes, a.vec != 0,
                                rowf, a.in, a.foff_in};
  l0.escapes(a, wk);
  ct::LdsLoad<kV, Gm::G> ll{lds};
  ct::LdsStore<kV, Gm::G, false> sl{lds};
  ct::LdsStore<kV, Gm::G, true> slf{lds};
  MaskStore<Gm::G> ms{lds, m2, a.k};
  GStore<LB2, true, true, decltype(destf)> sg{a.out + wk.blk * a.stride_out + wk.tile * a.tstride_out, a.ld_out, wk.lane0, a.lanes,
                                        a.vec != 0, destf, a.out, a.foff_out};
  sg.escapes(a, wk);
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<LB1, Gm::BM, kV, Gm::G, true>(tws, l0, ll, sl, ms);
  ct::dif<LB2, Gm::BM, kV, Gm::G, false>(tws, ll, ll, slf, sg);
}

// LDS storer of the product: natural index m1' of FNT_M pass B with
// sub = m2' -> times ahat[m2' + (M/256) m1'] (which carries M^-1); the lazy
// product is below 2^17 in magnitude.
template <int G>
struct AhatStore {
  uint32_t* lds;
  const uint32_t* t_ah;   // ahat[m2' + (M/256) m1'] by m1' (the workgroup's table)
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t pb, uint32_t g, int32_t (&x)[1 << B][kV]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t h = t_ah[pb + c * H];
#pragma unroll
      for (int v = 0; v < kV; ++v) x[c][v] = ct::mulw(x[c][v], h);
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
  uint32_t* t_ah = lds + Gm::LDS_BYTES / 4;   // read after the first barrier
  uint32_t* t_tw = t_ah + 256;                // w_M^-(m2' m2'')
  for (uint32_t t = threadIdx.x; t < 256u; t += kNT) {
    t_ah[t] = gptr(a.ahat_t)[(m2p << 8) + t];
    t_tw[t] = gptr(a.twsplit)[(m2p << 8) + t];
  }
  auto rowf = [&](uint32_t i1p, uint32_t& w) -> uint64_t {
    w = 0;
    return (uint64_t)i1p * rows2 + m2p;
  };
  auto destf = [&](uint32_t m2pp, uint32_t& w) -> uint64_t {
    w = t_tw[m2pp];
    return (uint64_t)m2p * 256u + m2pp;
  };
  GLoad<8, kScratch, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.tile * a.tstride_in, a.ld_in, wk.lane0,
                                        a.lanes, a.vec != 0, rowf, a.in, a.foff_in};
  l0.escapes(a, wk);
  ct::LdsLoad<kV, Gm::G> ll{lds};
  ct::LdsStore<kV, Gm::G, false> sl{lds};
  ct::LdsStore<kV, Gm::G, true> slf{lds};
  AhatStore<Gm::G> ah{lds, t_ah};
  GStore<8, true, true, decltype(destf)> sg{a.out + wk.blk * a.stride_out + wk.tile * a.tstride_out, a.ld_out, wk.lane0, a.lanes,
                                      a.vec != 0, destf, a.out, a.foff_out};
  sg.escapes(a, wk);
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
  GLoad<LB, kScratch, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.tile * a.tstride_in, a.ld_in, wk.lane0,
                                         a.lanes, a.vec != 0, rowf, a.in, a.foff_in};
  l0.escapes(a, wk);
  ct::LdsLoad<kV, Gm::G> ll{lds};
  ct::LdsStore<kV, Gm::G, false> sl{lds};
  GStore<LB, false, false, decltype(destf)> sg{a.out + wk.blk * a.stride_out + wk.tile * a.tstride_out, a.ld_out, wk.lane0, a.lanes,
                                        a.vec != 0, destf};
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<LB, Gm::BM, kV, Gm::G, true>(tws, l0, ll, sl, sg);
}

// Encoder as one FNT_n of the zero-padded source, n = N1 * 256.  Pass A:
// rows i1 + N1 i2 (zero from k on), forward, times w_n^(i1 m2) -> scratch
// row i1*256 + m2.  R: k <= n / 2^R, so rows with i2 >= 2^(8-R) are zero
// and the first R stages only copy (GLoad REP).
template <int R>
__global__ void __launch_bounds__(kNT) k4_enc1(FourStepArgs a) {
  using Gm = Geo<8>;
  extern __shared__ uint32_t lds[];
  const Work wk = work_of(a);
  const uint32_t i1 = wk.sub, N1 = a.n >> 8;
  uint32_t* t_tw = lds + Gm::LDS_BYTES / 4;   // w_n^(i1 m2), read after the first barrier
  for (uint32_t t = threadIdx.x; t < 256u; t += kNT) t_tw[t] = gptr(a.twsplit)[(i1 << 8) + t];
  auto rowf = [&](uint32_t i2, uint32_t& w) -> uint64_t {
    w = 0;
    const uint32_t j = i1 + N1 * i2;
    return j < a.k ? (uint64_t)j : ~0ull;
  };
  auto destf = [&](uint32_t m2, uint32_t& w) -> uint64_t {
    w = t_tw[m2];
    return (uint64_t)i1 * 256u + m2;
  };
  GLoad<8, kZeros, decltype(rowf), R> l0{a.in + wk.blk * a.stride_in + wk.tile * a.tstride_in, a.ld_in, wk.lane0,
                                         a.lanes, a.vec != 0, rowf};
  ct::LdsLoad<kV, Gm::G> lm{lds};
  ct::LdsStore<kV, Gm::G, false> sm{lds};
  GStore<8, false, true, decltype(destf)> sl{a.out + wk.blk * a.stride_out + wk.tile * a.tstride_out, a.ld_out, wk.lane0, a.lanes,
                                       a.vec != 0, destf, a.out, a.foff_out};
  sl.escapes(a, wk);
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
  GLoad<LB, kScratch, decltype(rowf)> l0{a.in + wk.blk * a.stride_in + wk.tile * a.tstride_in, a.ld_in, wk.lane0,
                                         a.lanes, a.vec != 0, rowf, a.in, a.foff_in};
  l0.escapes(a, wk);
  ct::LdsLoad<kV, Gm::G> lm{lds};
  ct::LdsStore<kV, Gm::G, false> sm{lds};
  GStore<LB, false, false, decltype(destf)> sl{a.out + wk.blk * a.stride_out + wk.tile * a.tstride_out, a.ld_out, wk.lane0, a.lanes,
                                       a.vec != 0, destf};
  using TW = typename Gm::TwType;
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  ct::dit<LB, Gm::BM, kV, Gm::G, false>(tws, l0, lm, sm, sl);
}

// First launch of a four-step call: clears the escape bitmaps of the call
// (up to three ranges of whole 16-byte vectors) before their writers run.
// The decoder's launch also lays out K1's weights and rows by sub-transform,
// so that each K1 workgroup reads its 256 pairs from one contiguous 2 KiB
// range instead of 512 words 4*n/256 bytes apart.
__global__ void __launch_bounds__(256) k_fs_prep(FsPrepArgs c) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    uint4* q = reinterpret_cast<uint4*>(c.p[j]);
    const uint64_t nv = c.words[j] / 4;
    for (uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x; t < nv; t += (uint64_t)gridDim.x * 256)
      q[t] = make_uint4(0, 0, 0, 0);
  }
  if (c.wr) {
    const uint32_t N1 = c.n >> 8;
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < c.n; t += gridDim.x * 256) {
      const uint32_t i1 = t >> 8, i2 = t & 255u, z = i1 + N1 * i2;
      const uint32_t w = gptr(c.wfull)[z];
      const uint32_t r = c.full ? z : gptr(c.ridx)[z];
      const u32x2 v = {w, w ? r : 0u};
      *(FNTRS_GLOBAL u32x2*)gptr(c.wr + 2 * (uint64_t)t) = v;
    }
  }
  if (c.ahat_t) {
    const uint32_t rows2 = c.M >> 8;
    for (uint32_t t = blockIdx.x * 256 + threadIdx.x; t < c.M; t += gridDim.x * 256)
      gptr(c.ahat_t)[t] = gptr(c.ahat)[(t >> 8) + rows2 * (t & 255u)];
  }
}

}  // namespace fs
}  // namespace fntrs
