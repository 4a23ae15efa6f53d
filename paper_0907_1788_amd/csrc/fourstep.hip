// Launches of the four-step kernels (fourstep.hpp) for n = 65536.
#include "fourstep.hpp"
#include "fourstep_launch.hpp"

namespace fntrs {

namespace {

template <class K>
hipError_t launch(K kernel, size_t lds, uint32_t blocks, const FourStepArgs& a, hipStream_t s) {
  (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(kernel, dim3(blocks), dim3(fs::kNT), lds, s, a);
  return hipGetLastError();
}

#define FNTRS_TRY(x)                    \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) return e_;    \
  } while (0)

}  // namespace

// Decoder for n = 65536 (and k = n) through two scratch buffers of n and M rows.
hipError_t fourstep_decode(const FourStepArgs& base, uint32_t batch, uint32_t* sa, uint32_t* sb, uint64_t lds_,
                           hipStream_t s) {
  const uint32_t tiles = base.tiles;
  const uint64_t ld = lds_;
  FourStepArgs a = base;
  // K1: recv -> sa (n rows)
  a.out = sa; a.ld_out = ld; a.stride_out = ld * a.n;
  a.subs = a.n >> 8;
  FNTRS_TRY(launch(fs::k4_dec1<8>, fs::Geo<8>::LDS_BYTES, tiles * a.subs * batch, a, s));
  if (base.k == base.n) {
    // erasure-free: the inverse transform's pass B writes the source
    FourStepArgs b = base;
    b.in = sa; b.ld_in = ld; b.stride_in = ld * a.n;
    b.subs = 256;
    b.M = base.n;
    return launch(fs::k4_dec4<8>, fs::Geo<8>::LDS_BYTES, tiles * b.subs * batch, b, s);
  }
  // K2: sa -> sb (M rows)
  FourStepArgs b = base;
  b.in = sa; b.ld_in = ld; b.stride_in = ld * a.n;
  b.out = sb; b.ld_out = ld; b.stride_out = ld * base.M;
  b.subs = 256;
  if (base.logm == 16)
    FNTRS_TRY(launch(fs::k4_dec2<8, 8>, fs::Geo<8>::LDS_BYTES, tiles * b.subs * batch, b, s));
  else
    FNTRS_TRY(launch(fs::k4_dec2<8, 7>, fs::Geo<8>::LDS_BYTES, tiles * b.subs * batch, b, s));
  // K3: sb -> sa (M rows)
  FourStepArgs c = base;
  c.in = sb; c.ld_in = ld; c.stride_in = ld * base.M;
  c.out = sa; c.ld_out = ld; c.stride_out = ld * a.n;
  c.subs = base.M >> 8;
  FNTRS_TRY(launch(fs::k4_dec3, fs::Geo<8>::LDS_BYTES, tiles * c.subs * batch, c, s));
  // K4: sa -> dst
  FourStepArgs d = base;
  d.in = sa; d.ld_in = ld; d.stride_in = ld * a.n;
  d.subs = 256;
  if (base.logm == 16) return launch(fs::k4_dec4<8>, fs::Geo<8>::LDS_BYTES, tiles * d.subs * batch, d, s);
  return launch(fs::k4_dec4<7>, fs::Geo<7>::LDS_BYTES, tiles * d.subs * batch, d, s);
}

// Encoder for K = n = 65536 through one scratch buffer of n rows.
hipError_t fourstep_encode(const FourStepArgs& base, uint32_t batch, uint32_t* sa, uint64_t lds_, hipStream_t s) {
  FourStepArgs a = base;
  a.out = sa; a.ld_out = lds_; a.stride_out = lds_ * a.n;
  a.subs = 256;
  FNTRS_TRY(launch(fs::k4_enc1, fs::Geo<8>::LDS_BYTES, base.tiles * a.subs * batch, a, s));
  FourStepArgs b = base;
  b.in = sa; b.ld_in = lds_; b.stride_in = lds_ * a.n;
  b.subs = 256;
  return launch(fs::k4_enc2, fs::Geo<8>::LDS_BYTES, base.tiles * b.subs * batch, b, s);
}

}  // namespace fntrs
