// Locator kernels: the position-only steps 1-3 of the interpolation of
// Sec. II-B, run once per erasure pattern and shared by every lane.
//
// Polynomials here are monic; a degree-d polynomial is stored as its d low
// coefficients (the leading 1 is implicit).
#pragma once
#include "lds_fnt.hpp"

namespace fntrs {

// x_i = r_n^(z_i) = 3^(z_i * 65536/n).
__device__ __forceinline__ uint32_t point_of(const uint32_t* tw, uint32_t z, int logn) {
  return tw[(z << (16 - logn)) & 0xFFFFu];
}

// Step 1, leaves of the product tree: group g multiplies the G linear factors
// (x - x_i), i in [gG, gG+G), one factor at a time (schoolbook; G <= 64).
__global__ void __launch_bounds__(64) k_loc_leaves(const uint32_t* __restrict__ pos, int logn, int G,
                                                   const uint32_t* __restrict__ tw,
                                                   uint32_t* __restrict__ out) {
  __shared__ uint32_t c[2][66];
  const int g = blockIdx.x;
  for (int j = threadIdx.x; j < 66; j += blockDim.x) { c[0][j] = (j == 0); c[1][j] = 0; }
  __syncthreads();
  int cur = 0;
  for (int i = 0; i < G; ++i) {
    const uint32_t x = point_of(tw, pos[g * G + i], logn);
    // (sum_j c_j x^j)(x - x_i): new_j = c_(j-1) - x_i c_j, degree i -> i+1
    for (int j = threadIdx.x; j <= i + 1; j += blockDim.x) {
      const uint32_t lo = j ? c[cur][j - 1] : 0u;
      c[cur ^ 1][j] = fsub(lo, fmul(x, c[cur][j]));
    }
    __syncthreads();
    cur ^= 1;
  }
  for (int j = threadIdx.x; j < G; j += blockDim.x) out[g * G + j] = c[cur][j];
}

// Step 1, one level of the product tree: pair p multiplies the monic degree-d
// polynomials a = x^d + a_lo and b = x^d + b_lo:
//   a b = x^(2d) + x^d (a_lo + b_lo) + a_lo b_lo,
// with a_lo b_lo (degree <= 2d-2) from three FNTs of size 2d (the
// transform-based product of Sec. II-B).  LDS holds one size-2d transform;
// the transform of a_lo is parked in `spec` (2d words per pair).
__global__ void __launch_bounds__(1024) k_loc_mul_level(const uint32_t* __restrict__ in, int logd,
                                                        const uint32_t* __restrict__ tw,
                                                        uint32_t* __restrict__ spec,
                                                        uint32_t* __restrict__ out) {
  extern __shared__ uint32_t lds[];
  const uint32_t d = 1u << logd, d2 = 2u * d;
  const uint32_t p = blockIdx.x;
  const uint32_t* a = in + (uint64_t)(2 * p) * d;
  const uint32_t* b = a + d;
  uint32_t* sp = spec + (uint64_t)p * d2;
  const uint32_t inv2d = 65537u - (65536u >> logd >> 1);   // (2d)^-1 = -2^16/(2d)
  for (uint32_t j = threadIdx.x; j < d2; j += blockDim.x) lds[j] = j < d ? a[j] : 0u;
  __syncthreads();
  lds_dif<1>(lds, 1, logd + 1, false, tw);
  for (uint32_t j = threadIdx.x; j < d2; j += blockDim.x) {
    sp[j] = lds[j];
    lds[j] = j < d ? b[j] : 0u;
  }
  __syncthreads();
  lds_dif<1>(lds, 1, logd + 1, false, tw);
  for (uint32_t j = threadIdx.x; j < d2; j += blockDim.x) lds[j] = fmul(lds[j], sp[j]);
  __syncthreads();
  lds_dit<1>(lds, 1, logd + 1, true, tw);
  uint32_t* o = out + (uint64_t)p * d2;
  for (uint32_t j = threadIdx.x; j < d2; j += blockDim.x) {
    uint32_t v = fmul(lds[j], inv2d);
    if (j >= d) v = fadd(v, fadd(a[j - d], b[j - d]));
    o[j] = v;
  }
}

// Step 2: A'(x) from the monic degree-k A (low coefficients a_0..a_(k-1)):
// coefficient j of A' is (j+1) a_(j+1), with a_k = 1.
__global__ void k_loc_derivative(const uint32_t* __restrict__ a, uint32_t k, uint32_t* __restrict__ da) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const uint32_t next = (j + 1 < k) ? a[j + 1] : 1u;
  da[j] = fmul(next, (j + 1) % 65537u);
}

// Evaluate c (K = 2^logK coefficients) at every N-th root of unity, N = K*cosets:
// value at r_N^(t + cosets*m) is FNT_K of (c_j r_N^(t j))_j at m (Sec. II-A,
// polynomial view of the FNT).  One workgroup per coset t.
__global__ void __launch_bounds__(1024) k_loc_eval(const uint32_t* __restrict__ c, int logK, int logN,
                                                   const uint32_t* __restrict__ tw,
                                                   uint32_t* __restrict__ vals) {
  extern __shared__ uint32_t lds[];
  const uint32_t K = 1u << logK, N = 1u << logN;
  const uint32_t t = blockIdx.x;
  const uint32_t cosets = N >> logK;
  for (uint32_t j = threadIdx.x; j < K; j += blockDim.x) {
    uint32_t v = c[j];
    if (t) v = fmul(v, tw[((t * j) & (N - 1)) << (16 - logN)]);
    lds[bitrev(j, logK)] = v;
  }
  __syncthreads();
  lds_dit<1>(lds, 1, logK, false, tw);
  for (uint32_t m = threadIdx.x; m < K; m += blockDim.x) vals[t + cosets * m] = lds[m];
}

// Step 3 and the weights of step 4: w_i = 1/A'(x_i), and the decoder weight
// -w_i x_i^(-1) (sign and index shift of step 5 folded in) scattered to the
// per-position tables: wfull[z_i] = -w_i x_i^(-1), ridx[z_i] = i.  wfull
// must be zero beforehand so that erased positions read as 0.
__global__ void k_loc_weights(const uint32_t* __restrict__ pos, const uint32_t* __restrict__ vals,
                              uint32_t k, int logn, const uint32_t* __restrict__ tw,
                              uint32_t* __restrict__ w, uint32_t* __restrict__ wfull,
                              uint32_t* __restrict__ ridx) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const uint32_t z = pos[i];
  const uint32_t wi = finv(vals[z]);
  const uint32_t xinv = tw[(65536u - ((z << (16 - logn)) & 0xFFFFu)) & 0xFFFFu];
  w[i] = wi;
  wfull[z] = fsub(0u, fmul(wi, xinv));
  ridx[z] = i;
}

// Â for step 6 with the inverse-transform factor M^-1 folded in (M = 2^logm
// is the cyclic length of the low product), in bit-reversed and in natural
// order.
__global__ void k_loc_ahat(const uint32_t* __restrict__ ahat, int logm, uint32_t* __restrict__ ahat_br,
                           uint32_t* __restrict__ ahat_s) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (1u << logm)) return;
  const uint32_t inv = 65537u - (65536u >> logm);           // (2^logm)^-1 = -2^(16-logm)
  const uint32_t v = fmul(ahat[i], inv);
  ahat_br[bitrev(i, logm)] = v;
  ahat_s[i] = v;
}

// Decoder tables when nothing is erased (k = n): weight n^-1, row z.
__global__ void k_loc_identity(uint32_t* __restrict__ wfull, uint32_t* __restrict__ ridx, uint32_t n,
                               uint32_t ninv) {
  const uint32_t z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= n) return;
  wfull[z] = ninv;
  ridx[z] = z;
}

// Fill k words with v.
__global__ void k_loc_fill(uint32_t* __restrict__ w, uint32_t k, uint32_t v) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) w[i] = v;
}

// n = 1 (and k = 1): encoding and decoding both copy the single symbol.
__global__ void k_copy_rows(const uint32_t* __restrict__ src, uint64_t stride_src, uint32_t* __restrict__ dst,
                            uint64_t stride_dst, uint32_t lanes, uint32_t batch, const uint32_t* __restrict__ scale) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (uint64_t)lanes * batch) return;
  const uint64_t b = i / lanes, l = i % lanes;
  const uint32_t v = src[b * stride_src + l];
  dst[b * stride_dst + l] = scale ? fmul(v, scale[0]) : v;
}

}  // namespace fntrs
