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

// Split twiddles of the four-step passes, laid out so that a workgroup reads
// its factors from one contiguous range.  The context's twiddle allocation
// holds tw (3^e), twi (3^-e), the stage tables (field.hpp), then for each
// N = 2^13 .. 2^16 (n, and the
// decoder's product length M >= n/2) four tables of N words: w_N^(i t) and
// w_N^-(i t) by [i < N/256][t < 256] (layout A), then the same by
// [i < 256][t < N/256] (layout B); w_N = 3^(65536/N).
constexpr int kSplitTwMinLog = kFourStepMinLog - 1;
constexpr size_t kSplitTwWords = 4 * ((size_t(1) << 17) - (size_t(1) << kSplitTwMinLog));
__host__ __device__ constexpr size_t split_tw_offset(int logN, bool layout_b, bool inv) {
  return kStageTwBase + kStageTwWords + 4 * ((size_t(1) << logN) - (size_t(1) << kSplitTwMinLog)) +
         (size_t(2 * (layout_b ? 1 : 0) + (inv ? 1 : 0)) << logN);
}

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
