// Host entry points of the four-step kernels (transforms of 2^14 .. 2^16 points).
#pragma once
#include <hip/hip_runtime.h>

#include "codec_args.hpp"
#include "kernel_args.hpp"

namespace fntrs {


// Lanes per tile of the four-step kernels.
#ifndef FNTRS_FS_TILE
#define FNTRS_FS_TILE 32
#endif
constexpr int kFourStepTile = FNTRS_FS_TILE;
// Transforms of 2^kFourStepMinLog points or more run as four-step passes:
// a single-pass tile of one such lane-transform fills the LDS with 1 or 2
// lanes, whose 4- or 8-byte row segments waste most of each HBM burst.
constexpr int kFourStepMinLog = 14;

// Decoder for n = 2^14 .. 2^16: `base` carries recv (in), dst (out), the tables and
// sizes (n, k, M, logn, logm, lanes, full, tiles, vec); sa (n rows) and sb
// (M rows) are scratch buffers [batch][rows][ld_scratch].
hipError_t fourstep_decode(const FourStepArgs& base, uint32_t batch, uint32_t* sa, uint32_t* sb,
                           uint64_t ld_scratch, hipStream_t s);
// Encoder for n = 2^14 .. 2^16 (one FNT_n of the zero-padded source): `base`
// carries src (in) and dst (out); sa is a scratch buffer of n rows per block.
hipError_t fourstep_encode(const FourStepArgs& base, uint32_t batch, uint32_t* sa, uint64_t ld_scratch,
                           hipStream_t s);

}  // namespace fntrs
