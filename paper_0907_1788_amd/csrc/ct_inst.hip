// One transform size of the compile-time kernels; built once per L with
// -DFNTRS_L=L (see build.py).
#include "ct_kernels.hpp"
#include "ct_launch.hpp"

#ifndef FNTRS_L
#error "FNTRS_L must be defined"
#endif

namespace fntrs {
namespace {

template <int L, int T, int NT, int V>
hipError_t enc_one(const EncodeArgs& a, uint32_t blocks, hipStream_t s) {
  constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
  static_assert(lds <= 163840, "tile exceeds LDS");
  lds_attr_once((const void*)ct::k_enc<L, T, NT, V>, lds);
  hipLaunchKernelGGL((ct::k_enc<L, T, NT, V>), dim3(blocks), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <int L, int D, int T, int NT, int V>
hipError_t dec_one(const DecodeArgs& a, uint32_t blocks, hipStream_t s) {
  constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
  static_assert(lds <= 163840, "tile exceeds LDS");
  lds_attr_once((const void*)ct::k_dec<L, D, T, NT, V>, lds);
  hipLaunchKernelGGL((ct::k_dec<L, D, T, NT, V>), dim3(blocks), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <int L, int T, int NT, int V>
hipError_t dec_t(int D, const DecodeArgs& a, uint32_t blocks, hipStream_t s) {
  if (D == -1) return dec_one<L, -1, T, NT, V>(a, blocks, s);
  if (D == 0) return dec_one<L, 0, T, NT, V>(a, blocks, s);
  if constexpr (L > 1) {
    if (D == 1) return dec_one<L, 1, T, NT, V>(a, blocks, s);
  }
  return hipErrorInvalidValue;
}

template <int L, int T, int NT, int V>
hipError_t enc_tab_one(const JobTable<EncodeArgs>& t, const uint32_t* tw, const uint32_t* twi, uint32_t grid,
                       hipStream_t s) {
  constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
  lds_attr_once((const void*)ct::k_enc_tab<L, T, NT, V>, lds);
  hipLaunchKernelGGL((ct::k_enc_tab<L, T, NT, V>), dim3(grid), dim3(NT), lds, s, t, tw, twi);
  return hipGetLastError();
}

template <int L, int D, int T, int NT, int V>
hipError_t dec_tab_one(const JobTable<DecodeArgs>& t, const uint32_t* tw, const uint32_t* twi, uint32_t grid,
                       hipStream_t s) {
  constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
  lds_attr_once((const void*)ct::k_dec_tab<L, D, T, NT, V>, lds);
  hipLaunchKernelGGL((ct::k_dec_tab<L, D, T, NT, V>), dim3(grid), dim3(NT), lds, s, t, tw, twi);
  return hipGetLastError();
}

template <int L, int T, int NT, int V>
hipError_t dec_tab_t(int D, const JobTable<DecodeArgs>& t, const uint32_t* tw, const uint32_t* twi, uint32_t grid,
                     hipStream_t s) {
  if (D == -1) return dec_tab_one<L, -1, T, NT, V>(t, tw, twi, grid, s);
  if (D == 0) return dec_tab_one<L, 0, T, NT, V>(t, tw, twi, grid, s);
  if constexpr (L > 1) {
    if (D == 1) return dec_tab_one<L, 1, T, NT, V>(t, tw, twi, grid, s);
  }
  return hipErrorInvalidValue;
}

// The pipelined decoder needs whole pass-0 items per thread and two passes.
template <int L, int T, int NT, int V>
constexpr bool pipe_ok() {
  using Gm = ct::Geo<L, T, NT, V>;
  return ct::pass0_per_thread<L, Gm::BM, Gm::G, NT>() >= 1 && ct::plan_np(L, Gm::BM) >= 2;
}

// The all-cosets encoder needs a first and a last pass.  It holds a tile's
// source rows in registers across the cosets, so it is used only where that
// costs neither a spill nor resident workgroups against k_enc (checked once
// per configuration).
template <int L, int T, int NT, int V>
constexpr bool cos_ok() {
  using Gm = ct::Geo<L, T, NT, V>;
  return L >= 2 && ct::plan_np(L, Gm::BM) >= 2;
}

template <class K>
bool kernel_spills(K kernel) {
  hipFuncAttributes at{};
  return hipFuncGetAttributes(&at, (const void*)kernel) != hipSuccess || at.localSizeBytes > 0;
}

template <int L, int T, int NT, int V>
bool enc_cos_pays() {
  constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
  if (kernel_spills(ct::k_enc_cos<L, T, NT, V>)) return false;
  int oc = 0, op = 0;
  lds_attr_once((const void*)ct::k_enc_cos<L, T, NT, V>, lds);
  lds_attr_once((const void*)ct::k_enc<L, T, NT, V>, lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&oc, ct::k_enc_cos<L, T, NT, V>, NT, lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&op, ct::k_enc<L, T, NT, V>, NT, lds) != hipSuccess)
    return false;
  return oc >= 1 && oc >= op;
}

template <int L, int T, int NT, int V>
hipError_t enc_cos_one(const EncodeArgs& a, uint32_t blocks, hipStream_t s) {
  if constexpr (cos_ok<L, T, NT, V>()) {
    static const bool pays = enc_cos_pays<L, T, NT, V>();
    if (!pays) return hipErrorNotSupported;
    constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
    lds_attr_once((const void*)ct::k_enc_cos<L, T, NT, V>, lds);
    hipLaunchKernelGGL((ct::k_enc_cos<L, T, NT, V>), dim3(blocks), dim3(NT), lds, s, a);
    return hipGetLastError();
  } else {
    return hipErrorNotSupported;
  }
}

template <int L, int T, int NT, int V>
bool enc_cos_tab_pays() {
  constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
  if (kernel_spills(ct::k_enc_cos_tab<L, T, NT, V>)) return false;
  int oc = 0, op = 0;
  lds_attr_once((const void*)ct::k_enc_cos_tab<L, T, NT, V>, lds);
  lds_attr_once((const void*)ct::k_enc_tab<L, T, NT, V>, lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&oc, ct::k_enc_cos_tab<L, T, NT, V>, NT, lds) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&op, ct::k_enc_tab<L, T, NT, V>, NT, lds) != hipSuccess)
    return false;
  return oc >= 1 && oc >= op;
}

template <int L, int T, int NT, int V>
hipError_t enc_cos_tab_one(const JobTable<EncodeArgs>& t, const uint32_t* tw, const uint32_t* twi, uint32_t grid,
                           hipStream_t s) {
  if constexpr (cos_ok<L, T, NT, V>()) {
    static const bool pays = enc_cos_tab_pays<L, T, NT, V>();
    if (!pays) return hipErrorNotSupported;
    constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
    lds_attr_once((const void*)ct::k_enc_cos_tab<L, T, NT, V>, lds);
    hipLaunchKernelGGL((ct::k_enc_cos_tab<L, T, NT, V>), dim3(grid), dim3(NT), lds, s, t, tw, twi);
    return hipGetLastError();
  } else {
    return hipErrorNotSupported;
  }
}

template <int L, int D, int T, int NT, int V>
hipError_t dec_pipe_one(const JobTable<DecodeArgs>& t, const DecodeArgs& one, const uint32_t* tw, const uint32_t* twi,
                        uint32_t grid, hipStream_t s) {
  if constexpr (pipe_ok<L, T, NT, V>()) {
    constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
    lds_attr_once((const void*)ct::k_dec_pipe<L, D, T, NT, V>, lds);
    hipLaunchKernelGGL((ct::k_dec_pipe<L, D, T, NT, V>), dim3(grid), dim3(NT), lds, s, t, one, tw, twi);
    return hipGetLastError();
  } else {
    return hipErrorNotSupported;
  }
}

template <int L, int T, int NT, int V>
hipError_t dec_pipe_t(int D, const JobTable<DecodeArgs>& t, const DecodeArgs& one, const uint32_t* tw,
                      const uint32_t* twi, uint32_t grid, hipStream_t s) {
  if (D == -1) return dec_pipe_one<L, -1, T, NT, V>(t, one, tw, twi, grid, s);
  if (D == 0) return dec_pipe_one<L, 0, T, NT, V>(t, one, tw, twi, grid, s);
  if constexpr (L > 1) {
    if (D == 1) return dec_pipe_one<L, 1, T, NT, V>(t, one, tw, twi, grid, s);
  }
  return hipErrorInvalidValue;
}

// A pipelined kernel that spills registers to scratch loses to the plain one:
// report it as unavailable.
template <class K>
int occupancy_no_spill(K kernel, int NT, size_t lds) {
  hipFuncAttributes at{};
  if (hipFuncGetAttributes(&at, (const void*)kernel) != hipSuccess || at.localSizeBytes > 0) return 0;
  int nb = 0;
  lds_attr_once((const void*)kernel, lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, NT, lds) != hipSuccess) return 0;
  return nb;
}

template <class K>
int occupancy(K kernel, int NT, size_t lds) {
  int nb = 0;
  lds_attr_once((const void*)kernel, lds);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, NT, lds) != hipSuccess) return 0;
  return nb;
}

template <int L, int T, int NT, int V>
int occ_t(int op, int D) {
  constexpr size_t lds = ct::Geo<L, T, NT, V>::LDS_BYTES;
  if (op == 3) {   // the all-cosets table encoder, where it exists and pays
    if constexpr (cos_ok<L, T, NT, V>()) {
      static const bool pays = enc_cos_tab_pays<L, T, NT, V>();
      if (pays) return occupancy(ct::k_enc_cos_tab<L, T, NT, V>, NT, lds);
    }
    return 0;
  }
  if (op == 2) {
    if constexpr (pipe_ok<L, T, NT, V>()) {
      if (D == -1) return occupancy_no_spill(ct::k_dec_pipe<L, -1, T, NT, V>, NT, lds);
      if (D == 0) return occupancy_no_spill(ct::k_dec_pipe<L, 0, T, NT, V>, NT, lds);
      if constexpr (L > 1) {
        if (D == 1) return occupancy_no_spill(ct::k_dec_pipe<L, 1, T, NT, V>, NT, lds);
      }
    }
    return 0;
  }
  if (op == 0) return occupancy(ct::k_enc_tab<L, T, NT, V>, NT, lds);
  if (D == -1) return occupancy(ct::k_dec_tab<L, -1, T, NT, V>, NT, lds);
  if (D == 0) return occupancy(ct::k_dec_tab<L, 0, T, NT, V>, NT, lds);
  if constexpr (L > 1) {
    if (D == 1) return occupancy(ct::k_dec_tab<L, 1, T, NT, V>, NT, lds);
  }
  return 0;
}

constexpr CtVariants kVar = ct_variants(FNTRS_L);

template <int I>
hipError_t enc_pick(CtCfg c, const EncodeArgs& a, uint32_t blocks, hipStream_t s) {
  if constexpr (I < 4 && kVar.enc[I < 4 ? I : 0].T != 0) {
    if (c.T == kVar.enc[I].T && c.NT == kVar.enc[I].NT && c.V == kVar.enc[I].V)
      return enc_one<FNTRS_L, kVar.enc[I].T, kVar.enc[I].NT, kVar.enc[I].V>(a, blocks, s);
    return enc_pick<I + 1>(c, a, blocks, s);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int I>
hipError_t dec_pick(CtCfg c, int D, const DecodeArgs& a, uint32_t blocks, hipStream_t s) {
  if constexpr (I < 4 && kVar.dec[I < 4 ? I : 0].T != 0) {
    if (c.T == kVar.dec[I].T && c.NT == kVar.dec[I].NT && c.V == kVar.dec[I].V)
      return dec_t<FNTRS_L, kVar.dec[I].T, kVar.dec[I].NT, kVar.dec[I].V>(D, a, blocks, s);
    return dec_pick<I + 1>(c, D, a, blocks, s);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int I>
hipError_t enc_tab_pick(CtCfg c, const JobTable<EncodeArgs>& t, const uint32_t* tw, const uint32_t* twi,
                        uint32_t grid, hipStream_t s) {
  if constexpr (I < 4 && kVar.enc[I < 4 ? I : 0].T != 0) {
    if (c.T == kVar.enc[I].T && c.NT == kVar.enc[I].NT && c.V == kVar.enc[I].V)
      return enc_tab_one<FNTRS_L, kVar.enc[I].T, kVar.enc[I].NT, kVar.enc[I].V>(t, tw, twi, grid, s);
    return enc_tab_pick<I + 1>(c, t, tw, twi, grid, s);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int I>
hipError_t dec_tab_pick(CtCfg c, int D, const JobTable<DecodeArgs>& t, const uint32_t* tw, const uint32_t* twi,
                        uint32_t grid, hipStream_t s) {
  if constexpr (I < 4 && kVar.dec[I < 4 ? I : 0].T != 0) {
    if (c.T == kVar.dec[I].T && c.NT == kVar.dec[I].NT && c.V == kVar.dec[I].V)
      return dec_tab_t<FNTRS_L, kVar.dec[I].T, kVar.dec[I].NT, kVar.dec[I].V>(D, t, tw, twi, grid, s);
    return dec_tab_pick<I + 1>(c, D, t, tw, twi, grid, s);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int I>
hipError_t enc_cos_pick(CtCfg c, const EncodeArgs& a, uint32_t blocks, hipStream_t s) {
  if constexpr (I < 4 && kVar.enc[I < 4 ? I : 0].T != 0) {
    if (c.T == kVar.enc[I].T && c.NT == kVar.enc[I].NT && c.V == kVar.enc[I].V)
      return enc_cos_one<FNTRS_L, kVar.enc[I].T, kVar.enc[I].NT, kVar.enc[I].V>(a, blocks, s);
    return enc_cos_pick<I + 1>(c, a, blocks, s);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int I>
hipError_t enc_cos_tab_pick(CtCfg c, const JobTable<EncodeArgs>& t, const uint32_t* tw, const uint32_t* twi,
                            uint32_t grid, hipStream_t s) {
  if constexpr (I < 4 && kVar.enc[I < 4 ? I : 0].T != 0) {
    if (c.T == kVar.enc[I].T && c.NT == kVar.enc[I].NT && c.V == kVar.enc[I].V)
      return enc_cos_tab_one<FNTRS_L, kVar.enc[I].T, kVar.enc[I].NT, kVar.enc[I].V>(t, tw, twi, grid, s);
    return enc_cos_tab_pick<I + 1>(c, t, tw, twi, grid, s);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int I>
hipError_t dec_pipe_pick(CtCfg c, int D, const JobTable<DecodeArgs>& t, const DecodeArgs& one, const uint32_t* tw,
                         const uint32_t* twi, uint32_t grid, hipStream_t s) {
  if constexpr (I < 4 && kVar.dec[I < 4 ? I : 0].T != 0) {
    if (c.T == kVar.dec[I].T && c.NT == kVar.dec[I].NT && c.V == kVar.dec[I].V)
      return dec_pipe_t<FNTRS_L, kVar.dec[I].T, kVar.dec[I].NT, kVar.dec[I].V>(D, t, one, tw, twi, grid, s);
    return dec_pipe_pick<I + 1>(c, D, t, one, tw, twi, grid, s);
  } else {
    return hipErrorInvalidValue;
  }
}

template <int I>
int occ_pick(CtCfg c, int op, int D) {
  if constexpr (I < 4) {
    constexpr CtCfg e = kVar.enc[I], d = kVar.dec[I];
    if constexpr (e.T != 0) {
      if ((op == 0 || op == 3) && c.T == e.T && c.NT == e.NT && c.V == e.V) return occ_t<FNTRS_L, e.T, e.NT, e.V>(op, D);
    }
    if constexpr (d.T != 0) {
      if ((op == 1 || op == 2) && c.T == d.T && c.NT == d.NT && c.V == d.V) return occ_t<FNTRS_L, d.T, d.NT, d.V>(op, D);
    }
    return occ_pick<I + 1>(c, op, D);
  } else {
    return 0;
  }
}

}  // namespace

#define FNTRS_CAT2(a, b) a##b
#define FNTRS_CAT(a, b) FNTRS_CAT2(a, b)

hipError_t FNTRS_CAT(ct_enc_launch_, FNTRS_L)(CtCfg c, const EncodeArgs& a, uint32_t blocks, hipStream_t s) {
  return enc_pick<0>(c, a, blocks, s);
}

hipError_t FNTRS_CAT(ct_dec_launch_, FNTRS_L)(CtCfg c, int D, const DecodeArgs& a, uint32_t blocks, hipStream_t s) {
  return dec_pick<0>(c, D, a, blocks, s);
}

hipError_t FNTRS_CAT(ct_enc_tab_launch_, FNTRS_L)(CtCfg c, const JobTable<EncodeArgs>& t, const uint32_t* tw,
                                                  const uint32_t* twi, uint32_t grid, hipStream_t s) {
  return enc_tab_pick<0>(c, t, tw, twi, grid, s);
}

hipError_t FNTRS_CAT(ct_dec_tab_launch_, FNTRS_L)(CtCfg c, int D, const JobTable<DecodeArgs>& t, const uint32_t* tw,
                                                  const uint32_t* twi, uint32_t grid, hipStream_t s) {
  return dec_tab_pick<0>(c, D, t, tw, twi, grid, s);
}

hipError_t FNTRS_CAT(ct_enc_cos_tab_launch_, FNTRS_L)(CtCfg c, const JobTable<EncodeArgs>& t, const uint32_t* tw,
                                                      const uint32_t* twi, uint32_t grid, hipStream_t s) {
  return enc_cos_tab_pick<0>(c, t, tw, twi, grid, s);
}

hipError_t FNTRS_CAT(ct_enc_cos_launch_, FNTRS_L)(CtCfg c, const EncodeArgs& a, uint32_t blocks, hipStream_t s) {
  return enc_cos_pick<0>(c, a, blocks, s);
}

hipError_t FNTRS_CAT(ct_dec_pipe_launch_, FNTRS_L)(CtCfg c, int D, const JobTable<DecodeArgs>& t,
                                                   const DecodeArgs& one, const uint32_t* tw, const uint32_t* twi,
                                                   uint32_t grid, hipStream_t s) {
  return dec_pipe_pick<0>(c, D, t, one, tw, twi, grid, s);
}

int FNTRS_CAT(ct_tab_occupancy_, FNTRS_L)(CtCfg c, int op, int D) { return occ_pick<0>(c, op, D); }

}  // namespace fntrs
