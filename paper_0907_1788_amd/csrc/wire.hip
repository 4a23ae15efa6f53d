// 16-bit transport of encoding symbols (Sec. II-B): every residue of GF(65537)
// but 65536 is a 16-bit value, and the positions of 65536 travel in the
// symbol's header.  A symbol is one row of `lanes` residues.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "host.hpp"

namespace fntrs {
namespace {

constexpr int kWireThreads = 256;   // one workgroup per row, four waves
constexpr uint32_t kMaxWireLanes = 65536;

// Row r of block b: lanes go out as their low 16 bits; the lanes holding
// 65536 are listed in ascending order (up to cap of them; count is the true
// number).  A wave ballot and the popcount of the lower lanes give each
// escape its slot, the wave totals in LDS give each wave its offset.
__global__ void __launch_bounds__(kWireThreads) k_pack16(const uint32_t* __restrict__ in, uint64_t ld_in,
                                                         uint64_t stride_in, uint32_t rows, uint32_t lanes,
                                                         uint16_t* __restrict__ out, uint64_t ld_out,
                                                         uint64_t stride_out, uint32_t* __restrict__ count,
                                                         uint32_t* __restrict__ pos, uint32_t cap) {
  __shared__ uint32_t wave_n[kWireThreads / 64];
  const uint32_t row = blockIdx.x;                      // b * rows + r
  const uint64_t b = row / rows, r = row % rows;
  const uint32_t* src = in + b * stride_in + r * ld_in;
  uint16_t* dst = out + b * stride_out + r * ld_out;
  const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  uint32_t base = 0;
  for (uint32_t l0 = 0; l0 < lanes; l0 += kWireThreads) {
    const uint32_t l = l0 + threadIdx.x;
    const uint32_t v = l < lanes ? src[l] : 0u;
    if (l < lanes) dst[l] = (uint16_t)(v & 0xFFFFu);
    const bool esc = l < lanes && v == 65536u;
    const uint64_t mask = __ballot(esc);
    if (lane == 0) wave_n[wave] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t off = base;
    for (uint32_t w = 0; w < wave; ++w) off += wave_n[w];
    if (esc) {
      const uint32_t slot = off + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
      if (slot < cap) pos[(uint64_t)row * cap + slot] = l;
    }
    uint32_t total = 0;
    for (uint32_t w = 0; w < kWireThreads / 64; ++w) total += wave_n[w];
    base += total;
    __syncthreads();   // wave_n is rewritten by the next chunk
  }
  if (threadIdx.x == 0) count[row] = base;
}

// Inverse: the listed lanes (the first min(count, cap)) become 65536 again,
// through a bitmask of the row in LDS; the other lanes are widened.
__global__ void __launch_bounds__(kWireThreads) k_unpack16(const uint16_t* __restrict__ in, uint64_t ld_in,
                                                           uint64_t stride_in, uint32_t rows, uint32_t lanes,
                                                           const uint32_t* __restrict__ count,
                                                           const uint32_t* __restrict__ pos, uint32_t cap,
                                                           uint32_t* __restrict__ out, uint64_t ld_out,
                                                           uint64_t stride_out) {
  __shared__ uint32_t bits[kMaxWireLanes / 32];
  const uint32_t row = blockIdx.x;
  const uint64_t b = row / rows, r = row % rows;
  const uint16_t* src = in + b * stride_in + r * ld_in;
  uint32_t* dst = out + b * stride_out + r * ld_out;
  const uint32_t words = (lanes + 31) / 32;
  for (uint32_t w = threadIdx.x; w < words; w += kWireThreads) bits[w] = 0u;
  __syncthreads();
  const uint32_t nesc = min(count[row], cap);
  for (uint32_t i = threadIdx.x; i < nesc; i += kWireThreads) {
    const uint32_t l = pos[(uint64_t)row * cap + i];
    if (l < lanes) atomicOr(&bits[l / 32], 1u << (l % 32));
  }
  __syncthreads();
  for (uint32_t l = threadIdx.x; l < lanes; l += kWireThreads)
    dst[l] = ((bits[l / 32] >> (l % 32)) & 1u) ? 65536u : (uint32_t)src[l];
}

int check_wire(fntrs_ctx* c, const void* in, size_t ld_in, size_t stride_in, uint32_t rows, uint32_t lanes,
               uint32_t batch, const void* out, size_t ld_out, size_t stride_out, const uint32_t* count,
               const uint32_t* pos, uint32_t cap) {
  if (rows < 1 || lanes < 1 || batch < 1) return fail(c, FNTRS_E_INVAL, "rows, lanes and batch must be >= 1");
  if (lanes > kMaxWireLanes) return fail(c, FNTRS_E_INVAL, "lanes=%u above %u", lanes, kMaxWireLanes);
  if ((uint64_t)rows * batch > 0x7fffffffull) return fail(c, FNTRS_E_INVAL, "rows x batch too large");
  if (!in || !out || !count || (cap && !pos)) return fail(c, FNTRS_E_INVAL, "null pointer");
  if (ld_in < lanes || ld_out < lanes) return fail(c, FNTRS_E_INVAL, "ld smaller than lanes");
  if (batch > 1 && (stride_in < (size_t)(rows - 1) * ld_in + lanes || stride_out < (size_t)(rows - 1) * ld_out + lanes))
    return fail(c, FNTRS_E_INVAL, "block strides overlap consecutive blocks");
  return FNTRS_OK;
}

}  // namespace
}  // namespace fntrs

using namespace fntrs;

extern "C" {

int fntrs_pack16(fntrs_ctx* c, const uint32_t* in, size_t ld_in, size_t stride_in, uint32_t rows, uint32_t lanes,
                 uint32_t batch, uint16_t* out, size_t ld_out, size_t stride_out, uint32_t* esc_count,
                 uint32_t* esc_pos, uint32_t esc_cap, void* stream) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (int rc = check_wire(c, in, ld_in, stride_in, rows, lanes, batch, out, ld_out, stride_out, esc_count, esc_pos,
                          esc_cap))
    return rc;
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
  DeviceGuard g(c->device);
  hipLaunchKernelGGL(k_pack16, dim3(rows * batch), dim3(kWireThreads), 0, (hipStream_t)stream, in, (uint64_t)ld_in,
                     (uint64_t)stride_in, rows, lanes, out, (uint64_t)ld_out, (uint64_t)stride_out, esc_count,
                     esc_pos, esc_cap);
  HIP_TRY(c, hipGetLastError());
  return FNTRS_OK;
}

int fntrs_unpack16(fntrs_ctx* c, const uint16_t* in, size_t ld_in, size_t stride_in, uint32_t rows, uint32_t lanes,
                   uint32_t batch, const uint32_t* esc_count, const uint32_t* esc_pos, uint32_t esc_cap,
                   uint32_t* out, size_t ld_out, size_t stride_out, void* stream) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (int rc = check_wire(c, in, ld_in, stride_in, rows, lanes, batch, out, ld_out, stride_out, esc_count, esc_pos,
                          esc_cap))
    return rc;
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
  DeviceGuard g(c->device);
  hipLaunchKernelGGL(k_unpack16, dim3(rows * batch), dim3(kWireThreads), 0, (hipStream_t)stream, in,
                     (uint64_t)ld_in, (uint64_t)stride_in, rows, lanes, esc_count, esc_pos, esc_cap, out,
                     (uint64_t)ld_out, (uint64_t)stride_out);
  HIP_TRY(c, hipGetLastError());
  return FNTRS_OK;
}

}  // extern "C"
