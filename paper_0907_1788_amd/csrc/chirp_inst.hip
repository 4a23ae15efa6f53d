// The fused chirp kernel of one product length 2^FNTRS_L (<= 2^13), in the
// decoder's default tile configuration of that size; built once per size
// (see build.py).
#include "chirp_kernels.hpp"
#include "ct_launch.hpp"

#ifndef FNTRS_L
#error "FNTRS_L must be defined"
#endif

namespace fntrs {

#define FNTRS_CHIRP_CAT2(a, b) a##b
#define FNTRS_CHIRP_CAT(a, b) FNTRS_CHIRP_CAT2(a, b)

// Launch over `blocks` = lane tiles x blocks; the tile's lanes in *tile.
hipError_t FNTRS_CHIRP_CAT(chirp_launch_, FNTRS_L)(const ChirpArgs& a, uint32_t blocks, hipStream_t s) {
  constexpr int L = FNTRS_L;
  constexpr CtCfg cfg = ct_variants(L).dec[0];
  using Gm = ct::Geo<L, cfg.T, cfg.NT, cfg.V>;
  constexpr size_t lds = Gm::LDS_BYTES;
  lds_attr_once((const void*)ct::k_chirp<L, cfg.T, cfg.NT, cfg.V>, lds);
  hipLaunchKernelGGL((ct::k_chirp<L, cfg.T, cfg.NT, cfg.V>), dim3(blocks), dim3(cfg.NT), lds, s, a);
  return hipGetLastError();
}

uint32_t FNTRS_CHIRP_CAT(chirp_tile_, FNTRS_L)() { return (uint32_t)ct_variants(FNTRS_L).dec[0].T; }

}  // namespace fntrs
