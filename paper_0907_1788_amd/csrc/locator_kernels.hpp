// Locator kernels: the position-only steps 1-3 of the interpolation of
// Sec. II-B, run once per erasure pattern and shared by every lane.
//
// Polynomials here are monic; a degree-d polynomial is stored as its d low
// coefficients (the leading 1 is implicit).
#pragma once
#include "ct_kernels.hpp"
#include "lds_fnt.hpp"
#include "kernel_args.hpp"

namespace fntrs {

// x_i = r_n^(z_i) = 3^(z_i * 65536/n).
__device__ __forceinline__ uint32_t point_of(const uint32_t* tw, uint32_t z, int logn) {
  return tw[(z << (16 - logn)) & 0xFFFFu];
}


// Pattern owning index x of a batch stage: the last i with start[i] <= x.
__device__ __forceinline__ uint32_t loc_find(const uint32_t* start, uint32_t count, uint32_t x) {
  uint32_t lo = 0, hi = count;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (start[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Stage 0, one thread per word: copy the positions into the state, clear the
// weights (an erased position must read weight 0).  Nothing erased (k = n):
// the decoder is the inverse FNT_n with factor n^-1, weight n^-1 and row z at
// every position, and A = x^n - 1.
__global__ void k_locb_prep(const LocDesc* __restrict__ D, const uint32_t* __restrict__ start, uint32_t count) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= start[count]) return;
  const uint32_t i = loc_find(start, count, x);
  const LocDesc& d = D[i];
  const uint32_t j = x - start[i];   // j < kr + n
  if (j < d.kr) {
    d.pos[j] = d.zin[j];
    if (d.kr == d.n) {
      d.A[j] = j == 0 ? 65536u : 0u;
      if (j == 0) d.A[d.kr] = 1u;
    }
  } else {
    const uint32_t z = j - d.kr;
    if (d.kr == d.n) {
      d.wfull[z] = 65537u - (65536u >> d.logn);
      d.ridx[z] = z;
    } else {
      d.wfull[z] = 0u;
    }
  }
}

// Step 1, leaves of the product tree: workgroup g of a pattern builds the
// product of the G linear factors (x - x_i), i in [gG, gG+G) (G <= 64), as
// its own small product tree in LDS: round h pairs monic degree-h
// polynomials a = x^h + a_lo, b = x^h + b_lo into
//   a b = x^(2h) + x^h (a_lo + b_lo) + a_lo b_lo,
// one output coefficient per thread (schoolbook, at most h terms), so the
// G points are read in one round and the tree takes log2(G) barriers.
__global__ void __launch_bounds__(64) k_locb_leaves(const LocDesc* __restrict__ D, const uint32_t* __restrict__ start,
                                                    uint32_t count, const uint32_t* __restrict__ tw) {
  __shared__ uint32_t c[2][64];
  const uint32_t i = loc_find(start, count, blockIdx.x);
  const LocDesc& d = D[i];
  const uint32_t g = blockIdx.x - start[i];
  const int G = (int)d.G;
  const int t = (int)threadIdx.x;
  // the leaves: monic degree 1, low coefficient -x_i; the points past the
  // received ones are roots at 0 (the tree then yields A(x) x^(k - kr))
  if (t < G) c[0][t] = g * G + t < d.kr ? fsub(0u, point_of(tw, d.zin[g * G + t], d.logn)) : 0u;
  __syncthreads();
  int cur = 0;
  for (int h = 1; h < G; h <<= 1) {
    if (t < G) {
      const uint32_t* a = &c[cur][(t / (2 * h)) * 2 * h];
      const uint32_t* b = a + h;
      const int j = t % (2 * h);
      uint32_t acc = j >= h ? fadd(a[j - h], b[j - h]) : 0u;
      const int lo = j - h + 1 > 0 ? j - h + 1 : 0, hi = j < h - 1 ? j : h - 1;
      for (int s2 = lo; s2 <= hi; ++s2) acc = fadd(acc, fmul(a[s2], b[j - s2]));
      c[cur ^ 1][t] = acc;
    }
    __syncthreads();
    cur ^= 1;
  }
  if (t < G) d.t0[g * G + t] = c[cur][t];
}

// Step 1, level `lev` of the product tree (degree d = G 2^lev): pair p of a
// pattern multiplies the monic degree-d polynomials a = x^d + a_lo and
// b = x^d + b_lo:
//   a b = x^(2d) + x^d (a_lo + b_lo) + a_lo b_lo,
// with a_lo b_lo (degree <= 2d-2) from three FNTs of size 2d (the
// transform-based product of Sec. II-B).  LDS holds one size-2d transform;
// the transform of a_lo is parked in `spec` (2d words per pair).  Levels
// alternate between the t0 and t1 buffers.
__global__ void __launch_bounds__(1024) k_locb_level(const LocDesc* __restrict__ D, const uint32_t* __restrict__ start,
                                                     uint32_t count, int logd, int lev,
                                                     const uint32_t* __restrict__ tw) {
  extern __shared__ uint32_t lds[];
  const uint32_t i = loc_find(start, count, blockIdx.x);
  const LocDesc& dd = D[i];
  const uint32_t p = blockIdx.x - start[i];
  const uint32_t d = 1u << logd, d2 = 2u * d;
  const uint32_t* in = (lev & 1) ? dd.t1 : dd.t0;
  uint32_t* outp = (lev & 1) ? dd.t0 : dd.t1;
  const uint32_t* a = in + (uint64_t)(2 * p) * d;
  const uint32_t* b = a + d;
  uint32_t* sp = dd.spec + (uint64_t)p * d2;
  const uint32_t inv2d = 65537u - (65536u >> logd >> 1);   // (2d)^-1 = -2^16/(2d)
  // The copies between global memory and LDS take kU words per thread at a
  // time, global reads first (see lds_fnt.hpp).  Word j of a round is
  // j0 + u*nt; the reads of words past the end are clamped to j0.
  const uint32_t nt = blockDim.x;
  for (uint32_t j0 = threadIdx.x; j0 < d2; j0 += kU * nt) {
    uint32_t v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt;
      v[u] = j < d ? gptr(a)[j] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (j0 + u * nt < d2) lds[j0 + u * nt] = v[u];
  }
  __syncthreads();
  lds_dif<1>(lds, 1, logd + 1, false, tw);
  for (uint32_t j0 = threadIdx.x; j0 < d2; j0 += kU * nt) {
    uint32_t v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt;
      v[u] = j < d ? gptr(b)[j] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt;
      if (j < d2) {
        gptr(sp)[j] = lds[j];
        lds[j] = v[u];
      }
    }
  }
  __syncthreads();
  lds_dif<1>(lds, 1, logd + 1, false, tw);
  for (uint32_t j0 = threadIdx.x; j0 < d2; j0 += kU * nt) {
    uint32_t v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt;
      v[u] = gptr(sp)[j < d2 ? j : j0];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt;
      if (j < d2) lds[j] = fmul(lds[j], v[u]);
    }
  }
  __syncthreads();
  lds_dit<1>(lds, 1, logd + 1, true, tw);
  uint32_t* o = outp + (uint64_t)p * d2;
  for (uint32_t j0 = threadIdx.x; j0 < d2; j0 += kU * nt) {
    uint32_t hi[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt;
      hi[u] = (j < d2 && j >= d) ? fadd(gptr(a)[j - d], gptr(b)[j - d]) : 0u;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt;
      if (j < d2) {
        uint32_t v = fmul(lds[j], inv2d);
        if (j >= d) v = fadd(v, hi[u]);
        gptr(o)[j] = v;
      }
    }
  }
}

// Step 2, one thread per coefficient of the tree (k of them): A (monic,
// degree kr) into the state -- the tree holds A(x) x^(k - kr), so a_j is its
// coefficient j + k - kr -- and A'(x): coefficient j of A' is (j+1) a_(j+1),
// with a_kr = 1, and zero from kr on (the evaluation reads k coefficients).
__global__ void k_locb_derivative(const LocDesc* __restrict__ D, const uint32_t* __restrict__ start, uint32_t count) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= start[count]) return;
  const uint32_t i = loc_find(start, count, x);
  const LocDesc& d = D[i];
  const uint32_t j = x - start[i];
  const uint32_t shift = d.k - d.kr;
  if (j < d.kr) {
    const uint32_t next = (j + 1 < d.kr) ? d.poly[j + 1 + shift] : 1u;
    d.A[j] = d.poly[j + shift];
    d.spec[j] = fmul(next, (j + 1) % 65537u);
  } else {
    d.spec[j] = 0u;
  }
  if (j == 0) d.A[d.kr] = 1u;
}

// Evaluate a polynomial with K = 2^logK coefficients at every N-th root of
// unity, N = K * cosets: the value at r_N^(t + cosets m) is FNT_K of
// (c_j r_N^(t j))_j at m (Sec. II-A, polynomial view of the FNT).  One
// workgroup per coset t.  Every pattern of the launch has a tree of K
// points.  A pattern's first n/K workgroups evaluate A' at the n-th roots
// (step 3); the next M/K evaluate A mod x^kr at the M-th roots (the
// transform of A used by the low product of step 6).
__global__ void __launch_bounds__(1024) k_locb_eval(const LocDesc* __restrict__ D, const uint32_t* __restrict__ start,
                                                    uint32_t count, int logK, const uint32_t* __restrict__ tw) {
  extern __shared__ uint32_t lds[];
  const uint32_t i = loc_find(start, count, blockIdx.x);
  const LocDesc& d = D[i];
  uint32_t t = blockIdx.x - start[i];
  const uint32_t K = 1u << logK;
  const uint32_t ncos = d.n >> logK;
  const bool deriv = t < ncos;
  if (!deriv) t -= ncos;
  const int logN = deriv ? d.logn : d.logm;
  const uint32_t N = 1u << logN;
  const uint32_t cosets = N >> logK;
  const uint32_t* c = deriv ? d.spec : d.A;       // A' (zero from kr on) or A mod x^kr
  const uint32_t lim = deriv ? K : d.kr;
  uint32_t* vals = deriv ? d.vals : d.ahat;
  const uint32_t nt = blockDim.x;
  for (uint32_t j0 = threadIdx.x; j0 < K; j0 += kU * nt) {   // global reads of kU words first
    uint32_t v[kU], w[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt < K ? j0 + u * nt : j0;
      v[u] = j < lim ? gptr(c)[j] : 0u;
      w[u] = gptr(tw)[((t * j) & (N - 1)) << (16 - logN)];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t j = j0 + u * nt;
      if (j < K) lds[bitrev(j, logK)] = t ? fmul(v[u], w[u]) : v[u];
    }
  }
  __syncthreads();
  lds_dit<1>(lds, 1, logK, false, tw);
  for (uint32_t m = threadIdx.x; m < K; m += blockDim.x) vals[t + cosets * m] = lds[m];
}

// Step 3 and the weights of step 4, one thread per received position:
// w_i = 1/A'(x_i), and the decoder weight -w_i x_i^(-1) (sign and index
// shift of step 5 folded in) scattered to the per-position tables:
// wfull[z_i] = -w_i x_i^(-1), ridx[z_i] = i.
__global__ void k_locb_weights(const LocDesc* __restrict__ D, const uint32_t* __restrict__ start, uint32_t count,
                               const uint32_t* __restrict__ tw) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= start[count]) return;
  const uint32_t i = loc_find(start, count, x);
  const LocDesc& d = D[i];
  const uint32_t q = x - start[i];
  const uint32_t z = d.pos[q];
  const uint32_t wi = finv(d.vals[z]);
  const uint32_t xinv = tw[(65536u - ((z << (16 - d.logn)) & 0xFFFFu)) & 0xFFFFu];
  d.w[q] = wi;
  d.wfull[z] = fsub(0u, fmul(wi, xinv));
  d.ridx[z] = q;
}

// Â for step 6 with the inverse-transform factor M^-1 folded in (M = 2^logm
// is the cyclic length of the low product), in bit-reversed and in natural
// order; one thread per value.
__global__ void k_locb_ahat(const LocDesc* __restrict__ D, const uint32_t* __restrict__ start, uint32_t count) {
  const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= start[count]) return;
  const uint32_t i = loc_find(start, count, x);
  const LocDesc& d = D[i];
  const uint32_t q = x - start[i];
  const uint32_t inv = 65537u - (65536u >> d.logm);   // (2^logm)^-1 = -2^(16-logm)
  const uint32_t v = fmul(d.ahat[q], inv);
  d.ahat_br[bitrev(q, d.logm)] = v;
  d.ahat_s[q] = v;
}

// ---------------------------------------------------------------- short codes
// Every step of the locator for one pattern of a short code in one workgroup
// (codes of at most kLocSmallN positions, so trees of at most kLocSmallN/2
// points): the product tree in LDS with schoolbook products (level h of a
// K-point tree costs K h products, h < K), A' at the n-th roots by K-point
// transforms, one coset at a time, and the transform of A for step 6 -- steps 1-3 and
// the tables of steps 4 and 6 of Sec. II-B without the launches and global
// round trips of the staged kernels above.  The state written is the same.
// Patterns with nothing erased take the staged path.
constexpr uint32_t kLocSmallN = 1024;
constexpr int kLocSmallNT = 512;

// zin: the pattern's received positions (a global pointer, or the array of
// a by-value argument).
template <class Z>
__device__ __forceinline__ void locb_small(const LocDesc& d, const Z& zin, const uint32_t* __restrict__ tw) {
  __shared__ uint32_t tree[2][kLocSmallN / 2];
  __shared__ uint32_t spec[kLocSmallN];   // A', then the transform of A
  __shared__ uint32_t vals[kLocSmallN];   // A' at the n-th roots
  __shared__ uint32_t buf[kLocSmallN / 2];
  const uint32_t n = d.n, K = d.k, kr = d.kr;
  const uint32_t t = threadIdx.x, nt = blockDim.x;
  // positions into the state; an erased position must read weight 0
  for (uint32_t j = t; j < n; j += nt) d.wfull[j] = 0u;
  for (uint32_t j = t; j < kr; j += nt) d.pos[j] = zin[j];
  // step 1: the tree of the K linear factors (x - x_i); the points past the
  // received ones are roots at 0, so the root holds A(x) x^(K - kr).  Round
  // h pairs monic degree-h polynomials a = x^h + a_lo, b = x^h + b_lo into
  // a b = x^(2h) + x^h (a_lo + b_lo) + a_lo b_lo, one coefficient a thread.
  for (uint32_t j = t; j < K; j += nt) tree[0][j] = j < kr ? fsub(0u, point_of(tw, zin[j], d.logn)) : 0u;
  __syncthreads();
  int cur = 0;
  for (uint32_t h = 1; h < K; h <<= 1) {
    for (uint32_t j = t; j < K; j += nt) {
      const uint32_t* a = &tree[cur][(j / (2 * h)) * 2 * h];
      const uint32_t* b = a + h;
      const uint32_t jj = j % (2 * h);
      uint32_t acc = jj >= h ? fadd(a[jj - h], b[jj - h]) : 0u;
      const uint32_t lo = jj >= h ? jj - h + 1 : 0u, hi = jj < h ? jj : h - 1;
      // four independent sums, so that their LDS reads issue together
      uint32_t acc1 = 0u, acc2 = 0u, acc3 = 0u, s2 = lo;
      for (; s2 + 3 <= hi; s2 += 4) {
        acc = fadd(acc, fmul(a[s2], b[jj - s2]));
        acc1 = fadd(acc1, fmul(a[s2 + 1], b[jj - s2 - 1]));
        acc2 = fadd(acc2, fmul(a[s2 + 2], b[jj - s2 - 2]));
        acc3 = fadd(acc3, fmul(a[s2 + 3], b[jj - s2 - 3]));
      }
      for (; s2 <= hi; ++s2) acc = fadd(acc, fmul(a[s2], b[jj - s2]));
      tree[cur ^ 1][j] = fadd(fadd(acc, acc1), fadd(acc2, acc3));
    }
    __syncthreads();
    cur ^= 1;
  }
  // step 2: A (monic, degree kr) into the state, and A' = sum (j+1) a_(j+1) x^j
  const uint32_t* poly = tree[cur];
  const uint32_t shift = K - kr;
  for (uint32_t j = t; j < K; j += nt) {
    if (j < kr) {
      const uint32_t next = j + 1 < kr ? poly[j + 1 + shift] : 1u;
      d.A[j] = poly[j + shift];
      spec[j] = fmul(next, j + 1);
    } else {
      spec[j] = 0u;
    }
  }
  if (t == 0) d.A[kr] = 1u;
  __syncthreads();
  // step 3: A' at every n-th root: the value at r_n^(c + cosets m) is FNT_K
  // of (a'_j r_n^(c j))_j at m (Sec. II-A, polynomial view of the FNT)
  const int logK = 31 - __clz(K);
  const uint32_t cosets = n >> logK;
  for (uint32_t c = 0; c < cosets; ++c) {
    for (uint32_t j = t; j < K; j += nt)
      buf[bitrev(j, logK)] = c ? fmul(spec[j], tw[((c * j) & (n - 1)) << (16 - d.logn)]) : spec[j];
    __syncthreads();
    lds_dit<1>(buf, 1, logK, false, tw);
    for (uint32_t m = t; m < K; m += nt) vals[c + cosets * m] = buf[m];
    __syncthreads();
  }
  // step 4: w_i = 1/A'(x_i), and the decoder weight -w_i x_i^(-1) (sign and
  // index shift of step 5) and row i at position z_i
  for (uint32_t q = t; q < kr; q += nt) {
    const uint32_t z = zin[q];
    const uint32_t wi = finv(vals[z]);
    const uint32_t xinv = tw[(65536u - ((z << (16 - d.logn)) & 0xFFFFu)) & 0xFFFFu];
    d.w[q] = wi;
    d.wfull[z] = fsub(0u, fmul(wi, xinv));
    d.ridx[z] = q;
  }
  // step 6 table: A mod x^kr at the M-th roots; unscaled in ahat, times M^-1
  // in natural and bit-reversed order
  const int logm = d.logm;
  const uint32_t M = 1u << logm;
  for (uint32_t j = t; j < M; j += nt) spec[bitrev(j, logm)] = j < kr ? poly[j + shift] : 0u;
  __syncthreads();
  lds_dit<1>(spec, 1, logm, false, tw);
  const uint32_t inv = 65537u - (65536u >> logm);   // (2^logm)^-1 = -2^(16-logm)
  for (uint32_t q = t; q < M; q += nt) {
    const uint32_t u = spec[q];
    const uint32_t v = fmul(u, inv);
    d.ahat[q] = u;
    d.ahat_br[bitrev(q, logm)] = v;
    d.ahat_s[q] = v;
  }
}

__global__ void __launch_bounds__(kLocSmallNT) k_locb_small(const LocDesc* __restrict__ D,
                                                            const uint32_t* __restrict__ tw) {
  const LocDesc& d = D[blockIdx.x];
  locb_small(d, d.zin, tw);
}

// One pattern whose descriptor and positions come by value: no upload, and
// no wait for one, in front of the kernel.
__global__ void __launch_bounds__(kLocSmallNT) k_locb_small1(LocSmallOne a, const uint32_t* __restrict__ tw) {
  locb_small(a.d, a.z, tw);
}

// ---------------------------------------------------------------- large
// transforms of the locator on the lane-tile engine (ctfnt.hpp) with one
// lane: radix-32 passes, one item per thread per pass (2^L / 32 threads,
// 64..1024), in place of the radix-4 LDS loops above: product-tree levels
// with transforms of 2^12 points and up (at 2^11 the radix-4 kernel is as
// fast), evaluations with K >= 2^11.
constexpr int kLocLevelCtMin = 12;
constexpr int kLocEvalCtMin = 11;

template <int L>
__host__ __device__ constexpr int loc_nt() {
  return (1 << (L - 5)) < 64 ? 64 : ((1 << (L - 5)) > 1024 ? 1024 : (1 << (L - 5)));
}
template <int L>
using LocGeo = ct::Geo<L, 1, loc_nt<L>(), 1>;

// First DIF pass over a monic polynomial's d = 2^(L-1) low coefficients,
// zero-padded to 2d: positions base + c*H with H = 2^(L-B); the upper half
// of an item (c >= 2^(B-1)) is exactly the padding.
struct PolyLoad {
  const uint32_t* a;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t, int32_t (&x)[1 << B][1]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) x[c][0] = c < (1 << (B - 1)) ? (int32_t)gptr(a)[base + c * H] : 0;
  }
};

// Last DIF pass of the first factor: its transform, canonical, parked in
// global scratch at its LDS position (the second factor's last pass has the
// same item layout, so each thread reads back what it wrote).
struct ParkStore {
  uint32_t* sp;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t, int32_t (&x)[1 << B][1]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) gptr(sp)[base + c * H] = ct::canon(x[c][0]);
  }
};

// Last DIT pass of the product: coefficient m (natural) of a_lo b_lo times
// (2d)^-1, plus a_(m-d) + b_(m-d) for m >= d (the c >= 2^(B-1) half).
struct LevelOut {
  uint32_t* o;
  const uint32_t* a;
  const uint32_t* b;
  uint32_t inv2d;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t, int32_t (&x)[1 << B][1]) {
    constexpr uint32_t D = H << (B - 1);
    uint32_t hi[1 << B];
#pragma unroll
    for (int c = 0; c < (1 << B); ++c)
      hi[c] = c < (1 << (B - 1)) ? 0u : fadd(gptr(a)[base + c * H - D], gptr(b)[base + c * H - D]);
#pragma unroll
    for (int c = 0; c < (1 << B); ++c)
      gptr(o)[base + c * H] = fadd(ct::canon(ct::mulc(ct::canon(x[c][0]), inv2d)), hi[c]);
  }
};

// k_locb_level for transforms of 2^L = 2d points: DIF of a_lo (parked), DIF
// of b_lo times the parked transform (in LDS), DIT back to the coefficients.
template <int L>
__global__ void __launch_bounds__(loc_nt<L>()) k_locb_level_ct(const LocDesc* __restrict__ D,
                                                             const uint32_t* __restrict__ start, uint32_t count,
                                                             int lev, const uint32_t* tw, const uint32_t* twi) {
  using Gm = LocGeo<L>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, tw, twi);
  __syncthreads();   // the first DIF pass reads the top stages' twiddles at once
  const uint32_t i = loc_find(start, count, blockIdx.x);
  const LocDesc& dd = D[i];
  const uint32_t p = blockIdx.x - start[i];
  constexpr uint32_t d = 1u << (L - 1), d2 = 2 * d;
  const uint32_t* in = (lev & 1) ? dd.t1 : dd.t0;
  uint32_t* outp = (lev & 1) ? dd.t0 : dd.t1;
  const uint32_t* a = in + (uint64_t)(2 * p) * d;
  const uint32_t* b = a + d;
  uint32_t* sp = dd.spec + (uint64_t)p * d2;
  ct::LdsLoad<1, 1> ll{lds};
  ct::LdsStore<1, 1, false> sl{lds};
  ct::LdsStore<1, 1, true> slf{lds};
  PolyLoad la{a}, lb{b};
  ParkStore park{sp};
  ct::ProductStore<1, 1> prod{lds, sp};
  LevelOut out{outp + (uint64_t)p * d2, a, b, 65537u - (65536u >> (L - 1) >> 1)};
  ct::dif<L, Gm::BM, 1, 1, false>(tws, la, ll, slf, park);
  ct::dif<L, Gm::BM, 1, 1, false>(tws, lb, ll, slf, prod);
  ct::dit<L, Gm::BM, 1, 1, true>(tws, ll, ll, sl, out);
}

// k_locb_eval for K = 2^LK: the encoder's work item on a one-lane codeword
// (the polynomial's K coefficients as K source rows, N = 2^logN points, one
// workgroup per coset t of N / K).
template <int LK>
__global__ void __launch_bounds__(loc_nt<LK>()) k_locb_eval_ct(const LocDesc* __restrict__ D,
                                                             const uint32_t* __restrict__ start, uint32_t count,
                                                             const uint32_t* tw, const uint32_t* twi) {
  using Gm = LocGeo<LK>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = ct::make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, tw, twi);
  const uint32_t i = loc_find(start, count, blockIdx.x);
  const LocDesc& d = D[i];
  uint32_t t = blockIdx.x - start[i];
  const uint32_t ncos = d.n >> LK;
  const bool deriv = t < ncos;
  if (!deriv) t -= ncos;
  const int logN = deriv ? d.logn : d.logm;
  EncodeArgs e{};
  e.src = deriv ? d.spec : d.A;    // A' or A mod x^kr (rows from e.k on read as zero)
  e.ld_src = 1;
  e.dst = deriv ? d.vals : d.ahat;
  e.ld_dst = 1;
  e.tw = tw;
  e.twi = twi;
  e.n = 1u << logN;
  e.k = deriv ? 1u << LK : d.kr;
  e.lanes = 1;
  e.logn = logN;
  e.logK = LK;
  e.tiles = 1;
  e.cosets = e.n >> LK;
  ct::enc_item<LK, 1, loc_nt<LK>(), 1>(e, t, lds, tws);
}

// ---------------------------------------------------------------- one large
// pattern: its top product-tree level and its evaluations as transforms
// spread over the four-step kernels (one lane), with these two pointwise
// kernels around them.
// x[i] = x[i] * y[i], i < count.
__global__ void k_loc_mul(uint32_t* __restrict__ x, const uint32_t* __restrict__ y, uint32_t count) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) x[i] = fmul(x[i], y[i]);
}

// The top level's product from the forward transform F of the product of
// the two halves' transforms: a_lo b_lo = F at negated indices / 2d, plus
// x^d (a_lo + b_lo) (monic factors: a b = x^(2d) + x^d (a_lo + b_lo) + a_lo b_lo).
__global__ void k_loc_combine(const uint32_t* __restrict__ F, const uint32_t* __restrict__ a,
                              const uint32_t* __restrict__ b, uint32_t* __restrict__ out, uint32_t d,
                              uint32_t inv2d) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= 2 * d) return;
  const uint32_t v = fmul(F[(2 * d - m) & (2 * d - 1)], inv2d);
  out[m] = m >= d ? fadd(v, fadd(a[m - d], b[m - d])) : v;
}

// ---------------------------------------------------------------- logarithms
// Steps 1-3 of Sec. II-B for one large pattern without the product tree.
// With x_z = r^z (r = r_n = 3^e, e = 65536/n) and R the k received
// positions, every value the decoder needs is a product of differences of
// points, and r^j - r^z = r^z (r^(j-z) - 1).  Taking discrete logarithms to
// base 3 (mod 65536, the order of the multiplicative group),
//   log A(x_j)   = S + C[j]            for j not in R,
//   log A'(x_z)  = S - e z + C[z]      for z in R (the factor z' = z left out),
// with S = e sum_{z in R} z and C[j] = sum_{z in R} l((j - z) mod n), where
// l(d) = log(r^d - 1) for d != 0 and l(0) = 0.  C is one cyclic convolution
// of the indicator of R with l.  It is exact over GF(65537) bit plane by bit
// plane: plane b of C counts the z in R whose l(j - z) has bit b set, at most
// k < 65537, so C mod 2^16 = sum_b 2^b count_b.  The tables FNT_n(plane_b(l))
// are fixed per n; a pattern costs the transform of its indicator, a product
// with the 16 planes, their 16 transforms back (a forward FNT read at negated
// indices, times n^-1) and one pass over the n positions.  From the values:
//   w_z = 1/A'(x_z),  the decoder weight -w_z x_z^(-1),
//   FNT_M(A mod x^k) at q = A(x_(q n/M)) - r_M^(q k)   (A monic of degree k, M <= n),
//   and the coefficients of A by one more transform of its n values (deg A = k < n).

// Indicator of R and the per-position tables: ind[j] = 1 for a received
// position j (rank q in the ascending list zin: pos[q] = j, ridx[j] = q),
// else 0.  Workgroup b covers positions [256 b, 256 b + 256), whose ranks
// are [bstart[b], bstart[b+1]) (from the host, which holds the positions).
__global__ void __launch_bounds__(256) k_conv_mark(const uint32_t* __restrict__ zin, const uint32_t* __restrict__ bstart,
                                                   uint32_t* __restrict__ ind, uint32_t* __restrict__ pos,
                                                   uint32_t* __restrict__ ridx) {
  __shared__ uint32_t rank1[256];   // rank + 1 of the position, 0: erased
  const uint32_t t = threadIdx.x, j0 = blockIdx.x * 256u;
  rank1[t] = 0u;
  const uint32_t q0 = bstart[blockIdx.x], q1 = bstart[blockIdx.x + 1];
  __syncthreads();
  if (q0 + t < q1) rank1[zin[q0 + t] - j0] = q0 + t + 1u;
  __syncthreads();
  const uint32_t v = rank1[t], j = j0 + t;
  ind[j] = v ? 1u : 0u;
  if (v) {
    pos[v - 1u] = j;
    ridx[j] = v - 1u;
  }
}

// P[j][b] = F[j] T[j][b] for the 16 bit planes (four per thread).
__global__ void k_conv_mul(const uint32_t* __restrict__ F, const uint32_t* __restrict__ T, uint32_t* __restrict__ P,
                           uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;   // (j, quarter)
  if (i >= 4 * n) return;
  const uint32_t f = F[i >> 2];
  const u32x4 t = *(const FNTRS_GLOBAL u32x4*)gptr(T + 4 * (size_t)i);
  *(FNTRS_GLOBAL u32x4*)gptr(P + 4 * (size_t)i) = u32x4{fmul(f, t.x), fmul(f, t.y), fmul(f, t.z), fmul(f, t.w)};
}

// One thread per position j: C[j] from the 16 counts, then A(x_j) or the
// weights of j, and FNT_M(A mod x^k) where j is a multiple of n/M.
__global__ void k_conv_finish(ConvFinishArgs a) {
  const uint32_t n = 1u << a.logn, j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const uint32_t e = 65536u >> a.logn;
  const uint32_t ninv = 65537u - e;   // n^-1 = -2^(16 - logn)
  const u32x4* q = (const u32x4*)(a.Q + (size_t)((n - j) & (n - 1)) * 16);
  uint32_t C = 0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const u32x4 c = *(const FNTRS_GLOBAL u32x4*)gptr(q + v);
    C += (fmul(c.x, ninv) << (4 * v)) + (fmul(c.y, ninv) << (4 * v + 1)) + (fmul(c.z, ninv) << (4 * v + 2)) +
         (fmul(c.w, ninv) << (4 * v + 3));
  }
  uint32_t val = 0;
  if (a.ind[j]) {
    const uint32_t lg = (a.S - e * j + C) & 0xFFFFu;                         // log A'(x_j)
    a.w[a.ridx[j]] = a.tw[(65536u - lg) & 0xFFFFu];                         // 1/A'(x_j)
    a.wfull[j] = a.tw[(32768u - lg - e * j) & 0xFFFFu];                     // -x_j^(-1)/A'(x_j)
  } else {
    a.wfull[j] = 0u;
    val = a.tw[(a.S + C) & 0xFFFFu];                                        // A(x_j)
  }
  a.vals[j] = val;
  const int sh = a.logn - a.logm;   // n/M = 2^sh
  if ((j & ((1u << sh) - 1)) == 0) {
    const uint32_t m = j >> sh, M = 1u << a.logm;
    const uint32_t u = fsub(val, a.tw[((m * a.kr) & (M - 1)) << (16 - a.logm)]);   // minus r_M^(m k)
    const uint32_t v = fmul(u, 65537u - (65536u >> a.logm));
    a.ahat[m] = u;
    a.ahat_br[bitrev(m, a.logm)] = v;
    a.ahat_s[m] = v;
  }
}

// Coefficients of A from the forward FNT_n G of its n values: a_i = G[-i] / n,
// i < k, and the leading 1.
__global__ void k_conv_coef(const uint32_t* __restrict__ G, uint32_t* __restrict__ A, uint32_t kr, int logn) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > kr) return;
  const uint32_t n = 1u << logn;
  A[i] = i == kr ? 1u : fmul(G[(n - i) & (n - 1)], 65537u - (65536u >> logn));
}

// The decoder's (weight, row) pairs in the order its first pass reads them:
// wrb[2p] = wfull[z], wrb[2p+1] = its row (z for a full recv, else ridx[z];
// 0 where the weight is 0), z = bitrev(p) over logn bits.
__global__ void __launch_bounds__(256) k_dec_pairs(const uint32_t* __restrict__ wfull, const uint32_t* __restrict__ ridx,
                                                   uint32_t* __restrict__ wrb, uint32_t n, int logn, uint32_t full) {
  for (uint32_t p = blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256) {
    const uint32_t z = __brev(p) >> (32 - logn);
    const uint32_t w = gptr(wfull)[z];
    const uint32_t r = w ? (full ? z : gptr(ridx)[z]) : 0u;
    const u32x2 v = {w, r};
    *(FNTRS_GLOBAL u32x2*)gptr(wrb + 2 * (uint64_t)p) = v;
  }
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
