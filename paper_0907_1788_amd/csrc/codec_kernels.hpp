// Encoder and decoder kernels: one workgroup owns T lanes of one codeword
// block and runs every transform of that block on chip (LDS).
#pragma once
#include "lds_fnt.hpp"

namespace fntrs {

struct EncodeArgs {
  const uint32_t* src;
  uint64_t ld_src, stride_src;
  uint32_t* dst;
  uint64_t ld_dst, stride_dst;
  const uint32_t* tw;      // tw[e] = 3^e
  uint32_t n, k, lanes;
  int logn, logK;          // K = 2^logK >= k, K <= n: transform size
  uint32_t tiles, cosets;  // lane tiles per block, n / K
};

// Encoder, Sec. II-B: e_i = s(r_n^i).  Output row i = t + (n/K) m is the m-th
// output of FNT_K applied to (s_j r_n^(t j))_j: since r_n^(n/K) = r_K,
// s(r_n^(t + (n/K) m)) = sum_j (s_j r_n^(t j)) r_K^(m j).  One workgroup per
// (lane tile, coset t, block); rows j >= k are the zero padding.
template <int T>
__global__ void __launch_bounds__(256) k_encode(EncodeArgs a) {
  extern __shared__ uint32_t lds[];
  const int ldr = T;
  uint32_t bid = blockIdx.x;
  const uint32_t tile = bid % a.tiles;
  bid /= a.tiles;
  const uint32_t t = bid % a.cosets;
  const uint64_t blk = bid / a.cosets;
  const uint32_t lane0 = tile * T;
  const uint32_t K = 1u << a.logK;
  const uint32_t* src = a.src + blk * a.stride_src + lane0;
  uint32_t* dst = a.dst + blk * a.stride_dst + lane0;
  const int sh = 16 - a.logn;

  for (uint32_t q = threadIdx.x; q < K * T; q += blockDim.x) {
    const uint32_t l = q & (T - 1);
    const uint32_t j = q / T;
    uint32_t v = 0;
    if (j < a.k && lane0 + l < a.lanes) {
      v = src[(uint64_t)j * a.ld_src + l];
      if (t) v = fmul(v, a.tw[((t * j) & (a.n - 1)) << sh]);
    }
    lds[bitrev(j, a.logK) * ldr + l] = v;
  }
  __syncthreads();
  lds_dit<T>(lds, ldr, a.logK, false, a.tw);
  for (uint32_t q = threadIdx.x; q < K * T; q += blockDim.x) {
    const uint32_t l = q & (T - 1);
    const uint32_t m = q / T;
    if (lane0 + l < a.lanes)
      dst[(uint64_t)(t + a.cosets * m) * a.ld_dst + l] = lds[m * ldr + l];
  }
}

struct DecodeArgs {
  const uint32_t* recv;
  uint64_t ld_recv, stride_recv;
  uint32_t* dst;
  uint64_t ld_dst, stride_dst;
  const uint32_t* tw;
  const uint32_t* pos;      // k received positions, ascending
  const uint32_t* wp;       // per-position input weights (see k_decode)
  const uint32_t* ahat_br;  // FNT_2k of A's low part, bit-reversed, times (2k)^-1
  uint32_t n, k, lanes;
  int logn, logk;
  uint32_t full;            // recv holds n rows indexed by position
  uint32_t tiles;
};

// Decoder, Sec. II-B steps 4-6, for one (lane tile, block):
//   step 4  n_i = v_i / A'(x_i); the locator supplies wp_i = -r_n^(-z_i) / A'(x_i)
//           so that u_(z_i) = wp_i v_i already carries the sign and the shift
//           of step 5 (zero at erased positions);
//   step 5  S_j = -N'(r^(-j-1)) = sum_z u_z r^(-j z)  for j < k: one unscaled
//           inverse FNT_n of u (inputs placed in bit-reversed order, DIT);
//   step 6  P = (A S) mod x^k: FNT_2k of (S, 0) (DIF, bit-reversed output),
//           times FNT_2k(A mod x^k) / 2k (bit-reversed), inverse FNT_2k (DIT),
//           keep the first k coefficients.
// With k = n (nothing erased) the locator sets wp_i = n^-1 and the inverse
// FNT_n alone is the decoder (Sec. II-B, erasure-free case).
template <int T>
__global__ void __launch_bounds__(256) k_decode(DecodeArgs a) {
  extern __shared__ uint32_t lds[];
  const int ldr = T;
  uint32_t bid = blockIdx.x;
  const uint32_t tile = bid % a.tiles;
  const uint64_t blk = bid / a.tiles;
  const uint32_t lane0 = tile * T;
  const uint32_t n = a.n, k = a.k;
  const uint32_t* recv = a.recv + blk * a.stride_recv + lane0;
  uint32_t* dst = a.dst + blk * a.stride_dst + lane0;

  for (uint32_t q = threadIdx.x; q < n * T; q += blockDim.x) lds[q] = 0;   // ldr == T
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < k * T; q += blockDim.x) {
    const uint32_t l = q & (T - 1);
    const uint32_t i = q / T;
    const uint32_t z = a.pos[i];
    uint32_t v = 0;
    if (lane0 + l < a.lanes) v = recv[(uint64_t)(a.full ? z : i) * a.ld_recv + l];
    lds[bitrev(z, a.logn) * ldr + l] = fmul(v, a.wp[i]);
  }
  __syncthreads();
  lds_dit<T>(lds, ldr, a.logn, true, a.tw);

  if (k != n) {
    const int log2k = a.logk + 1;
    const uint32_t k2 = 2u * k;
    for (uint32_t q = k * T + threadIdx.x; q < k2 * T; q += blockDim.x) lds[q] = 0;
    __syncthreads();
    lds_dif<T>(lds, ldr, log2k, false, a.tw);
    for (uint32_t q = threadIdx.x; q < k2 * T; q += blockDim.x)
      lds[q] = fmul(lds[q], a.ahat_br[q / T]);
    __syncthreads();
    lds_dit<T>(lds, ldr, log2k, true, a.tw);
  }
  for (uint32_t q = threadIdx.x; q < k * T; q += blockDim.x) {
    const uint32_t l = q & (T - 1);
    const uint32_t j = q / T;
    if (lane0 + l < a.lanes) dst[(uint64_t)j * a.ld_dst + l] = lds[j * ldr + l];
  }
}

}  // namespace fntrs
