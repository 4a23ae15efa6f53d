// Launch entry points of the compile-time kernels.  Each transform size L
// lives in its own translation unit (ct_inst.hip built with -DFNTRS_L=L), so
// the sizes compile in parallel; the host reaches them through these tables.
#pragma once
#include <hip/hip_runtime.h>

#include "codec_args.hpp"

namespace fntrs {

// Kernel configurations instantiated for encode / decode at size 2^L: lane
// tile width T, threads per workgroup NT and lanes per thread V (T = 0 ends
// a list).  The first
// entry is the default; the autotuner may pick another.
// Sets a kernel's dynamic LDS limit on the current device once per (kernel,
// device): the runtime call would otherwise cost host time at every launch.
void lds_attr_once(const void* fn, size_t bytes);

struct CtCfg {
  int T, NT;
  int V = 0;   // lanes per thread; 0 = 4 when the tile allows, else T
};
struct CtVariants {
  CtCfg enc[4];
  CtCfg dec[4];
};

constexpr CtVariants ct_variants(int L) {
  switch (L) {
    case 9: return {{{32, 512}, {64, 512}, {8, 128}}, {{32, 512}, {64, 512}, {8, 128}}};
    case 10: return {{{16, 512}, {32, 512}}, {{16, 512}, {32, 512}}};
    case 11: return {{{8, 512}, {16, 512}}, {{8, 512}, {16, 512}}};
    case 12: return {{{8, 512}, {8, 1024}, {4, 512, 2}, {8, 1024, 2}}, {{8, 1024, 2}, {8, 512}, {4, 512}, {8, 1024}}};
    case 13: return {{{4, 1024}, {4, 512}}, {{4, 1024}, {4, 512}, {4, 512, 2}}};
    case 14: return {{{2, 512}}, {{2, 512}}};
    case 15: return {{{1, 512}}, {{1, 512}}};
    default: return {{{64, 512}, {128, 512}, {16, 128}}, {{64, 512}, {128, 512}, {16, 128}}};   // L <= 8
  }
}

// Narrow tile for calls too small to fill the device with the default one
// (one codeword of a few hundred lanes): more, shorter workgroups.  T = 0
// when the size has none.  Each is also listed in ct_variants.
constexpr CtCfg ct_small(int L) {
  return L <= 8 ? CtCfg{16, 128} : (L == 9 ? CtCfg{8, 128} : CtCfg{0, 0});
}

// Launches k_enc<L, T, NT> / k_dec<L, D, T, NT>; D in {-1 (k = n), 0, 1}.
// Returns hipErrorInvalidValue for a configuration that is not instantiated.
using CtEncLaunch = hipError_t (*)(CtCfg cfg, const EncodeArgs& a, uint32_t blocks, hipStream_t s);
using CtDecLaunch = hipError_t (*)(CtCfg cfg, int D, const DecodeArgs& a, uint32_t blocks, hipStream_t s);

// Batched (table) launches: a persistent grid of `grid` workgroups walks the
// work items of every job in the table (k_enc_tab / k_dec_tab).
using CtEncTabLaunch = hipError_t (*)(CtCfg cfg, const JobTable<EncodeArgs>& t, const uint32_t* tw,
                                      const uint32_t* twi, uint32_t grid, hipStream_t s);
using CtDecTabLaunch = hipError_t (*)(CtCfg cfg, int D, const JobTable<DecodeArgs>& t, const uint32_t* tw,
                                      const uint32_t* twi, uint32_t grid, hipStream_t s);
// Encoder with all cosets of a lane tile in one workgroup (k_enc_cos); blocks
// = lane tiles x batch.  hipErrorNotSupported when the configuration has none.
using CtEncCosLaunch = hipError_t (*)(CtCfg cfg, const EncodeArgs& a, uint32_t blocks, hipStream_t s);
// Batched all-cosets encoder (k_enc_cos_tab): work items are (lane tile,
// block); hipErrorNotSupported when the configuration has none or it does
// not pay (occupancy op 3 is then 0).
using CtEncCosTabLaunch = CtEncTabLaunch;
// Pipelined persistent decoder launch (k_dec_pipe): a table of jobs, or
// (t.jobs == nullptr) the single job `one` with t.total work items.
// hipErrorNotSupported when the configuration has no pipelined kernel.
using CtDecPipeLaunch = hipError_t (*)(CtCfg cfg, int D, const JobTable<DecodeArgs>& t, const DecodeArgs& one,
                                       const uint32_t* tw, const uint32_t* twi, uint32_t grid, hipStream_t s);
// Workgroups of a persistent kernel that fit on one CU at once (0 when the
// configuration is not instantiated or has no such kernel); op 0 = encode
// table, 1 = decode table, 2 = decode pipelined, 3 = all-cosets encode table.
using CtTabOccupancy = int (*)(CtCfg cfg, int op, int D);

#define FNTRS_CT_DECL(L)                                                                              \
  hipError_t ct_enc_launch_##L(CtCfg cfg, const EncodeArgs& a, uint32_t blocks, hipStream_t s);           \
  hipError_t ct_dec_launch_##L(CtCfg cfg, int D, const DecodeArgs& a, uint32_t blocks, hipStream_t s);    \
  hipError_t ct_enc_tab_launch_##L(CtCfg cfg, const JobTable<EncodeArgs>& t, const uint32_t* tw,          \
                                   const uint32_t* twi, uint32_t grid, hipStream_t s);                    \
  hipError_t ct_dec_tab_launch_##L(CtCfg cfg, int D, const JobTable<DecodeArgs>& t, const uint32_t* tw,   \
                                   const uint32_t* twi, uint32_t grid, hipStream_t s);                    \
  hipError_t ct_enc_cos_launch_##L(CtCfg cfg, const EncodeArgs& a, uint32_t blocks, hipStream_t s);         \
  hipError_t ct_enc_cos_tab_launch_##L(CtCfg cfg, const JobTable<EncodeArgs>& t, const uint32_t* tw,      \
                                       const uint32_t* twi, uint32_t grid, hipStream_t s);                \
  hipError_t ct_dec_pipe_launch_##L(CtCfg cfg, int D, const JobTable<DecodeArgs>& t, const DecodeArgs& one,\
                                    const uint32_t* tw, const uint32_t* twi, uint32_t grid, hipStream_t s); \
  int ct_tab_occupancy_##L(CtCfg cfg, int op, int D);
FNTRS_CT_DECL(1) FNTRS_CT_DECL(2) FNTRS_CT_DECL(3) FNTRS_CT_DECL(4) FNTRS_CT_DECL(5)
FNTRS_CT_DECL(6) FNTRS_CT_DECL(7) FNTRS_CT_DECL(8) FNTRS_CT_DECL(9) FNTRS_CT_DECL(10)
FNTRS_CT_DECL(11) FNTRS_CT_DECL(12) FNTRS_CT_DECL(13) FNTRS_CT_DECL(14) FNTRS_CT_DECL(15)
#undef FNTRS_CT_DECL

}  // namespace fntrs
