// Number-theoretic transforms over GF(65537) on tiles held in LDS.
//
// A tile is `rows` rows of T lanes, row r / lane l at buf[r*ldr + l]; every
// lane is an independent transform along the rows (the paper applies the
// code to every 16-bit lane of a packet, Sec. II-B).  Transforms have size
// m = 2^logm and use the root omega_m = 3^(65536/m) (Sec. II-B root choice)
// or its inverse; twiddles come from a table tw[e] = 3^e, e < 65536, so that
// omega_m^j = tw[j << (16 - logm)].
//
// Two in-place radix-2 orderings are provided (the divide-and-conquer FNT of
// Sec. II-A, written iteratively), both fusing two radix-2 stages per pass
// through LDS (a radix-4 step per thread):
//   dit: input in bit-reversed row order, output in natural order;
//   dif: input in natural order, output in bit-reversed order.
// Neither scales by m^(-1); callers fold that factor elsewhere.
#pragma once
#include "field.hpp"

namespace fntrs {

// Exponent of omega_(2^lg)^j in the 3^e table, negated for the inverse root.
__device__ __forceinline__ uint32_t tw_exp(uint32_t j, int lg, bool inv) {
  uint32_t e = (j << (16 - lg)) & 0xFFFFu;
  return inv ? ((65536u - e) & 0xFFFFu) : e;
}

// A thread takes its items of a pass kU at a time and reads all their
// twiddles (global table) before it touches LDS: the item loop is not
// unrolled, and a twiddle read placed after an LDS store through a generic
// pointer could not be moved above it, so every item would wait for its own
// read.
constexpr int kU = 4;

template <int T>
__device__ void lds_dit(uint32_t* buf, int ldr, int logm, bool inv,
                        const uint32_t* __restrict__ tw) {
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  const int m = 1 << logm;
  int s = 0;
  while (s < logm) {
    if (s + 1 < logm) {
      const int h = 1 << s;
      const int items = T * (m >> 2);
      for (int q0 = tid; q0 < items; q0 += kU * nt) {
        uint32_t w1[kU], w2[kU], w3[kU];
        int off[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int q = q0 + u * nt < items ? q0 + u * nt : q0;
          const int l = q & (T - 1);
          const int g = q / T;
          const int jp = g & (h - 1);
          off[u] = (((g >> s) << (s + 2)) | jp) * ldr + l;
          w1[u] = gptr(tw)[tw_exp(jp, s + 1, inv)];
          w2[u] = gptr(tw)[tw_exp(jp, s + 2, inv)];
          w3[u] = gptr(tw)[tw_exp(jp + h, s + 2, inv)];
        }
        const int st = h * ldr;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (q0 + u * nt >= items) break;
          uint32_t* p = buf + off[u];
          const uint32_t a0 = p[0], a1 = p[st], a2 = p[2 * st], a3 = p[3 * st];
          uint32_t t = fmul_tw(a1, w1[u]);
          const uint32_t b0 = fadd(a0, t), b1 = fsub(a0, t);
          t = fmul_tw(a3, w1[u]);
          const uint32_t b2 = fadd(a2, t), b3 = fsub(a2, t);
          t = fmul_tw(b2, w2[u]);
          p[0] = fadd(b0, t);
          p[2 * st] = fsub(b0, t);
          t = fmul_tw(b3, w3[u]);
          p[st] = fadd(b1, t);
          p[3 * st] = fsub(b1, t);
        }
      }
      s += 2;
    } else {
      const int h = 1 << s;
      const int items = T * (m >> 1);
      for (int q0 = tid; q0 < items; q0 += kU * nt) {
        uint32_t w1[kU];
        int off[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int q = q0 + u * nt < items ? q0 + u * nt : q0;
          const int l = q & (T - 1);
          const int g = q / T;
          const int jp = g & (h - 1);
          off[u] = (((g >> s) << (s + 1)) | jp) * ldr + l;
          w1[u] = gptr(tw)[tw_exp(jp, s + 1, inv)];
        }
        const int st = h * ldr;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (q0 + u * nt >= items) break;
          uint32_t* p = buf + off[u];
          const uint32_t a0 = p[0];
          const uint32_t t = fmul_tw(p[st], w1[u]);
          p[0] = fadd(a0, t);
          p[st] = fsub(a0, t);
        }
      }
      s += 1;
    }
    __syncthreads();
  }
}

template <int T>
__device__ void lds_dif(uint32_t* buf, int ldr, int logm, bool inv,
                        const uint32_t* __restrict__ tw) {
  const int nt = blockDim.x;
  const int tid = threadIdx.x;
  const int m = 1 << logm;
  int s = logm - 1;            // current stage has half-size 2^s
  while (s >= 0) {
    if (s >= 1) {
      // stages s (half 2H) and s-1 (half H), H = 2^(s-1)
      const int H = 1 << (s - 1);
      const int items = T * (m >> 2);
      for (int q0 = tid; q0 < items; q0 += kU * nt) {
        uint32_t w1[kU], w2[kU], w3[kU];
        int off[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int q = q0 + u * nt < items ? q0 + u * nt : q0;
          const int l = q & (T - 1);
          const int g = q / T;
          const int jp = g & (H - 1);
          off[u] = (((g >> (s - 1)) << (s + 1)) | jp) * ldr + l;
          w2[u] = gptr(tw)[tw_exp(jp, s + 1, inv)];
          w3[u] = gptr(tw)[tw_exp(jp + H, s + 1, inv)];
          w1[u] = gptr(tw)[tw_exp(jp, s, inv)];
        }
        const int st = H * ldr;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          if (q0 + u * nt >= items) break;
          uint32_t* p = buf + off[u];
          const uint32_t x0 = p[0], x1 = p[st], x2 = p[2 * st], x3 = p[3 * st];
          const uint32_t y0 = fadd(x0, x2), y2 = fmul_tw(fsub(x0, x2), w2[u]);
          const uint32_t y1 = fadd(x1, x3), y3 = fmul_tw(fsub(x1, x3), w3[u]);
          p[0] = fadd(y0, y1);
          p[st] = fmul_tw(fsub(y0, y1), w1[u]);
          p[2 * st] = fadd(y2, y3);
          p[3 * st] = fmul_tw(fsub(y2, y3), w1[u]);
        }
      }
      s -= 2;
    } else {
      const int items = T * (m >> 1);
      for (int q = tid; q < items; q += nt) {
        const int l = q & (T - 1);
        const int g = q / T;
        uint32_t* p = buf + (2 * g) * ldr + l;
        const uint32_t x0 = p[0], x1 = p[ldr];
        p[0] = fadd(x0, x1);
        p[ldr] = fsub(x0, x1);          // omega_2^0 = 1
      }
      s -= 1;
    }
    __syncthreads();
  }
}

}  // namespace fntrs
