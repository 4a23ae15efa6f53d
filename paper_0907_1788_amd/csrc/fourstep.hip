// Launches of the four-step kernels (fourstep.hpp) for n = 2^14 .. 2^16.
#include "ct_launch.hpp"
#include "fourstep.hpp"
#include "fourstep_launch.hpp"

namespace fntrs {

namespace {

uint32_t ilog2_u64(uint64_t v) {
  uint32_t l = 0;
  while ((v >> l) > 1) ++l;
  return l;
}

template <class K>
hipError_t launch(K kernel, size_t lds, uint32_t blocks, const FourStepArgs& a, hipStream_t s) {
  lds_attr_once((const void*)kernel, lds);
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(fs::kNT), lds, s, a);
  return hipGetLastError();
}

#define FNTRS_TRY(x)                    \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

// The call's first launch (fs::k_fs_prep): zeroes the escape bitmaps and lays
// out the decoder's tables.
hipError_t prepare_call(const FsPrepArgs& c, hipStream_t s) {
  const uint64_t words = c.words[0] + c.words[1] + c.words[2];
  const uint64_t items = std::max<uint64_t>(words / 4, c.wr ? c.n / 4 : 0);   // c.M <= c.n
  const uint32_t blocks = (uint32_t)std::min<uint64_t>(1024, (items + 255) / 256 + 1);
  hipLaunchKernelGGL(fs::k_fs_prep, dim3(blocks), dim3(256), 0, s, c);
  return hipGetLastError();
}

// Byte offsets of the escape bitmaps in a scratch buffer of batch*rows*lds_
// words (4 bytes per element): the 2-byte values and flag bytes of a use take
// the first 2.5 bytes per element, the bitmaps (rows*tiles/8 bytes per block
// each) start at 3 bytes per element.  The decoder's first buffer (n rows)
// then holds, from 3.5 bytes per element, K1's (weight, row) pairs (8n bytes)
// and K3's layout of the locator's transform (4M bytes).
uint64_t bitmap_at(uint32_t batch, uint64_t rows, uint64_t lds_) { return 3 * (uint64_t)batch * rows * lds_; }
uint64_t bitmap_bytes(uint32_t batch, uint32_t tiles, uint64_t rows) { return (uint64_t)batch * tiles * rows / 8; }

template <int LB>
hipError_t dec4(const FourStepArgs& a, uint32_t blocks, hipStream_t s) {
  return launch(fs::k4_dec4<LB>, fs::Geo<LB>::LDS_BYTES, blocks, a, s);
}

hipError_t dec4_any(int LB, const FourStepArgs& a, uint32_t blocks, hipStream_t s) {
  switch (LB) {
    case 5: return dec4<5>(a, blocks, s);
    case 6: return dec4<6>(a, blocks, s);
    case 7: return dec4<7>(a, blocks, s);
    case 8: return dec4<8>(a, blocks, s);
    default: return hipErrorInvalidValue;
  }
}

template <int LB1, int LB2>
hipError_t dec2(const FourStepArgs& a, uint32_t blocks, hipStream_t s) {
  return launch(fs::k4_dec2<LB1, LB2>, fs::lds_with_tables<LB1>(), blocks, a, s);
}

// K2 for pass-B size 2^LB1 (n / 256) and FNT_M pass-A size 2^LB2 (M / 256).
hipError_t dec2_any(int LB1, int LB2, const FourStepArgs& a, uint32_t blocks, hipStream_t s) {
  if (LB1 == 6 && LB2 == 5) return dec2<6, 5>(a, blocks, s);
  if (LB1 == 6 && LB2 == 6) return dec2<6, 6>(a, blocks, s);
  if (LB1 == 7 && LB2 == 6) return dec2<7, 6>(a, blocks, s);
  if (LB1 == 7 && LB2 == 7) return dec2<7, 7>(a, blocks, s);
  if (LB1 == 8 && LB2 == 7) return dec2<8, 7>(a, blocks, s);
  if (LB1 == 8 && LB2 == 8) return dec2<8, 8>(a, blocks, s);
  return hipErrorInvalidValue;
}

}  // namespace

// Decoder for n = 2^14 .. 2^16 (and k = n) through two scratch buffers of n
// and M rows.  n = N1 * 256: K1 runs the size-256 passes A of the inverse
// FNT_n, K2 its size-N1 passes B and the size-M/256 passes A of FNT_M, K3 the
// size-256 passes B of FNT_M, the product with the locator's transform and
// the size-256 passes A of the inverse FNT_M, K4 its size-M/256 passes B.
// sa holds batch*n*lds_ words and sb batch*M*lds_ (lds_ = tiles * kT), both
// used tile-major.
hipError_t fourstep_decode(const FourStepArgs& base, uint32_t batch, uint32_t* sa, uint32_t* sb, uint64_t lds_,
                           hipStream_t s) {
  const uint32_t tiles = base.tiles;
  if (base.logn < 14 || base.logn > 16) return hipErrorInvalidValue;
  if (base.k != base.n && (base.logm < kSplitTwMinLog || base.logm > base.logn)) return hipErrorInvalidValue;
  if (lds_ != (uint64_t)tiles * fs::kT) return hipErrorInvalidValue;
  const int LB1 = base.logn - 8;
  const uint64_t T = fs::kT;
  // scratch of `rows` rows, tile-major
  // (the flags of a buffer used with `rows` rows follow its 2-byte values)
  // order (fs::work_of): sub-transform first for the kernels that read
  // scratch and write scratch (K2, K3), pairs of sub-transforms then tiles
  // for K4, which writes the caller's rows.
  auto scr_in = [&](FourStepArgs& f, const uint32_t* p, uint64_t rows, uint64_t boff, uint32_t order) {
    f.in = p; f.ld_in = T; f.tstride_in = rows * T; f.stride_in = tiles * rows * T;
    f.foff_in = 2 * (uint64_t)batch * f.stride_in;
    f.boff_in = boff; f.rlog_in = ilog2_u64(rows);
    f.order = order;
  };
  // slog: log2 of the writer's row split (rows i*S + m)
  auto scr_out = [&](FourStepArgs& f, uint32_t* p, uint64_t rows, uint64_t boff, uint32_t slog) {
    f.out = p; f.ld_out = T; f.tstride_out = rows * T; f.stride_out = tiles * rows * T;
    f.foff_out = 2 * (uint64_t)batch * f.stride_out;
    f.boff_out = boff; f.rlog_out = ilog2_u64(rows); f.slog_out = slog;
  };
  const uint64_t n = base.n, M = base.M;
  // bitmaps: K1's rows and K3's rows in sa, K2's rows in sb
  const uint64_t bA1 = bitmap_at(batch, n, lds_), bA2 = bA1 + bitmap_bytes(batch, tiles, n);
  const uint64_t bB = bitmap_at(batch, M, lds_);
  const uint64_t bWR = 7 * (uint64_t)batch * n * lds_ / 2;   // 3.5 bytes per element: 8 n bytes
  const uint64_t bAH = bWR + 8 * n;                            // then K3's Â layout, 4 M bytes
  {
    FsPrepArgs cl{};
    cl.p[0] = (uint32_t*)((uint8_t*)sa + bA1);
    cl.words[0] = bitmap_bytes(batch, tiles, n) / 4;
    // K1's weights and rows by sub-transform, beyond the bitmaps
    cl.wr = (uint32_t*)((uint8_t*)sa + bWR);
    cl.wfull = base.wfull; cl.ridx = base.ridx; cl.n = base.n; cl.full = base.full;
    if (base.k != base.n) {
      cl.ahat_t = (uint32_t*)((uint8_t*)sa + bAH);
      cl.ahat = base.ahat; cl.M = base.M;
      cl.p[1] = (uint32_t*)((uint8_t*)sa + bA2);
      cl.words[1] = bitmap_bytes(batch, tiles, M) / 4;
      cl.p[2] = (uint32_t*)((uint8_t*)sb + bB);
      cl.words[2] = bitmap_bytes(batch, tiles, M) / 4;
    }
    FNTRS_TRY(prepare_call(cl, s));
  }
  FourStepArgs user = base;   // the caller's buffers are row-major
  user.tstride_in = T;
  user.tstride_out = T;
  // K1: recv -> sa (n rows)
  FourStepArgs a = user;
  scr_out(a, sa, n, bA1, 8);
  a.wr = (const uint32_t*)((const uint8_t*)sa + bWR);
  a.twsplit = base.tw + split_tw_offset(base.logn, false, true);
  a.subs = a.n >> 8;
  FNTRS_TRY(launch(fs::k4_dec1<8>, fs::lds_with_tables<8>(), tiles * a.subs * batch, a, s));
  if (base.k == base.n) {
    // erasure-free: the inverse transform's pass B writes the source
    FourStepArgs b = user;
    scr_in(b, sa, n, bA1, 2);
    b.subs = 256;
    b.M = base.n;
    return dec4_any(LB1, b, tiles * b.subs * batch, s);
  }
  const int LB2 = base.logm - 8;
  // K2: sa -> sb (M rows)
  FourStepArgs b = user;
  scr_in(b, sa, n, bA1, 1);
  scr_out(b, sb, M, bB, base.logm - 8);
  b.twsplit = base.tw + split_tw_offset(base.logm, true, false);
  b.subs = 256;
  FNTRS_TRY(dec2_any(LB1, LB2, b, tiles * b.subs * batch, s));
  // K3: sb -> sa (M rows)
  FourStepArgs c = user;
  scr_in(c, sb, M, bB, 1);
  scr_out(c, sa, M, bA2, 8);
  c.twsplit = base.tw + split_tw_offset(base.logm, false, true);
  c.ahat_t = (const uint32_t*)((const uint8_t*)sa + bAH);
  c.subs = base.M >> 8;
  FNTRS_TRY(launch(fs::k4_dec3, fs::lds_with_tables<8>(), tiles * c.subs * batch, c, s));
  // K4: sa -> dst
  FourStepArgs d = user;
  scr_in(d, sa, M, bA2, 2);
  d.subs = 256;
  return dec4_any(LB2, d, tiles * d.subs * batch, s);
}

// Encoder as one FNT_n of the zero-padded source, n = 2^14 .. 2^16, through
// one scratch buffer of batch*n*lds_ words (lds_ = tiles * kT), tile-major.
hipError_t fourstep_encode(const FourStepArgs& base, uint32_t batch, uint32_t* sa, uint64_t lds_, hipStream_t s) {
  if (base.logn < 14 || base.logn > 16) return hipErrorInvalidValue;
  if (lds_ != (uint64_t)base.tiles * fs::kT) return hipErrorInvalidValue;
  const uint64_t T = fs::kT, rows = base.n;
  FourStepArgs a = base;
  a.tstride_in = T;
  a.out = sa; a.ld_out = T; a.tstride_out = rows * T; a.stride_out = base.tiles * rows * T;
  a.foff_out = 2 * (uint64_t)batch * a.stride_out;   // the flags follow the 2-byte values
  const uint64_t bA = bitmap_at(batch, rows, lds_);
  a.boff_out = bA; a.rlog_out = base.logn; a.slog_out = 8;
  a.twsplit = base.tw + split_tw_offset(base.logn, false, false);
  {
    FsPrepArgs cl{};
    cl.p[0] = (uint32_t*)((uint8_t*)sa + bA);
    cl.words[0] = bitmap_bytes(batch, base.tiles, rows) / 4;
    FNTRS_TRY(prepare_call(cl, s));
  }
  a.subs = a.n >> 8;
  // zero-padded source: k <= n/4 or n/2 lets the first pass skip its first stages
  const uint32_t grid1 = base.tiles * a.subs * batch;
  if (4ull * base.k <= base.n) FNTRS_TRY(launch(fs::k4_enc1<2>, fs::lds_with_tables<8>(), grid1, a, s));
  else if (2ull * base.k <= base.n) FNTRS_TRY(launch(fs::k4_enc1<1>, fs::lds_with_tables<8>(), grid1, a, s));
  else FNTRS_TRY(launch(fs::k4_enc1<0>, fs::lds_with_tables<8>(), grid1, a, s));
  FourStepArgs b = base;
  b.in = sa; b.ld_in = T; b.tstride_in = rows * T; b.stride_in = base.tiles * rows * T;
  b.foff_in = 2 * (uint64_t)batch * b.stride_in;
  b.boff_in = bA; b.rlog_in = base.logn;
  // pairs of sub-transforms, then tiles: reads the scratch lines whole and
  // keeps neighbouring tiles of the output rows together
  b.order = 2;
  b.tstride_out = T;
  b.subs = 256;
  switch (base.logn) {
    case 14: return launch(fs::k4_enc2<6>, fs::Geo<6>::LDS_BYTES, base.tiles * b.subs * batch, b, s);
    case 15: return launch(fs::k4_enc2<7>, fs::Geo<7>::LDS_BYTES, base.tiles * b.subs * batch, b, s);
    default: return launch(fs::k4_enc2<8>, fs::Geo<8>::LDS_BYTES, base.tiles * b.subs * batch, b, s);
  }
}

}  // namespace fntrs
