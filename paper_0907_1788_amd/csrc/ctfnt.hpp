// FNT passes over GF(65537) with compile-time plans, for gfx950.
//
// A transform of size 2^L runs along the rows of a tile of T = V*G lanes
// (V lanes per thread, G lane groups); every lane is an independent
// transform (Sec. II-B).  The L radix-2 stages of the divide-and-conquer FNT
// (Sec. II-A) are grouped into passes of B stages; a thread loads one item
// -- the 2^B positions base + c*2^S0 of V lanes -- into registers, runs the
// B stages there and writes it back.  Pass radices, strides and twiddle
// strides are template constants, so every LDS offset inside an item is an
// immediate.
//
// Orders: dit_*: input bit-reversed, output natural;
//         dif_*: input natural, output bit-reversed.
//
// Lazy arithmetic.  Values are int32 congruent to the residue and kept below
// 2^23 in magnitude.  Since p = 2^16 + 1, 2^16 = -1 and 2^32 = 1, so a
// product y*w (|y| < 2^23, w < 2^16) split into its low 32-bit word and the
// bits above is congruent to hi + lo16 - hi16(lo): a twiddle product costs
// two 24-bit multiplies and two adds with no reduction of y, and lands in
// [-65663, 65662].  A DIT butterfly x +- w*y grows ranges only additively
// (x +- t); a trivial butterfly (w = 1) or a DIF sum x + y doubles them, so
// the stages that double are few per pass and values are folded
// (lo16 - (v >> 16), one SDWA subtract) when a pass that doubles stores them.
// fold(fold(v)) lies in [-1, 65536] and an unsigned min maps -1 to 65536,
// which gives the canonical residue stored to global memory.
#pragma once
#include <type_traits>

#include "field.hpp"

namespace fntrs {
namespace ct {

// ---------------------------------------------------------------- arithmetic
__device__ __forceinline__ int32_t fold1(int32_t a) { return (int32_t)(a & 0xFFFF) - (a >> 16); }

__device__ __forceinline__ uint32_t canon(int32_t a) { return min((uint32_t)fold1(fold1(a)), 65536u); }

// y * w mod p for loose y with |y| < 2^23 and a residue w in [0, 65536].
// The signed 24-bit multiplier gives the 48-bit product as a low word and a
// high part h (|h| <= 128); 2^32 = 1 mod p, so y w = h + lo16 - hi16(lo).
// Result in [-65663, 65663].  Two multiplies and two adds, no reduction of y.
__device__ __forceinline__ int32_t mulw(int32_t y, uint32_t w) {
  const int32_t ys = (y << 8) >> 8;            // states |y| < 2^23 (the multiplier reads 24 bits)
  const int32_t wsx = (int32_t)(w << 8) >> 8;  // and w < 2^23
  const int64_t m = (int64_t)ys * (int64_t)wsx;
  const uint32_t lo = (uint32_t)m;
  const int32_t hi = (int32_t)(m >> 32);
  return (int32_t)(lo & 0xFFFFu) - (int32_t)(lo >> 16) + hi;
}

// y * c mod p for canonical y and any residue c in [0, 65536] (65536*65536 =
// 2^32 wraps to 0 in 32 bits; 2^32 = 1 mod p, added back through the top bits).
__device__ __forceinline__ int32_t mulc(uint32_t yc, uint32_t c) {
  const uint32_t m = __umul24(yc, c);
  return (int32_t)(m & 0xFFFFu) - (int32_t)(m >> 16) + (int32_t)((yc & c) >> 16);
}

// Small roots for passes whose twiddles are compile-time constants:
// root(lg, j) = omega_(2^lg)^j = 3^(j * 2^(16-lg)).
struct RootTable {
  uint32_t f[64], i[64];   // 3^(1024 j), 3^(-1024 j), j < 64
};
__host__ __device__ constexpr uint32_t cmul(uint32_t a, uint32_t b) {
  return (uint32_t)((uint64_t)a * b % 65537u);
}
__host__ __device__ constexpr RootTable make_roots() {
  RootTable t{};
  uint32_t g = 1;
  for (int e = 0; e < 1024; ++e) g = cmul(g, 3);           // 3^1024
  uint32_t ginv = 1;
  for (int e = 0; e < 65536 - 1024; ++e) ginv = cmul(ginv, 3);  // 3^-1024
  uint32_t a = 1, b = 1;
  for (int j = 0; j < 64; ++j) {
    t.f[j] = a;
    t.i[j] = b;
    a = cmul(a, g);
    b = cmul(b, ginv);
  }
  return t;
}
constexpr RootTable kRoots = make_roots();

template <bool INV>
__device__ __forceinline__ constexpr uint32_t small_root(int lg, int j) {
  // lg <= 6: omega_(2^lg)^j = 3^(1024 * j * 2^(6-lg))
  return INV ? kRoots.i[(j << (6 - lg)) & 63] : kRoots.f[(j << (6 - lg)) & 63];
}

// ---------------------------------------------------------------- LDS tile
// Vector index u = pos*G + g (V words each); one padding vector every 16
// vectors: phys(u) = u + u/16.  For an item (positions base + c*H, B >= 4
// or H*G >= 16) phys(u0 + c*H*G) = phys(u0) + c*H*G + (c*H*G)/16, a constant
// offset, and the strided accesses of a pass fall in distinct banks.
__device__ __forceinline__ uint32_t phys(uint32_t u) { return u + (u >> 4); }

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Renumber them so that consecutive logical ids run on the same XCD:
// neighbouring lane tiles, which share cache lines of every row, then meet
// in one L2 instead of each fetching whole lines from HBM.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nb) {
  const uint32_t xcd = bid & 7u, local = bid >> 3;
  const uint32_t per = nb >> 3, rem = nb & 7u;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}
__host__ __device__ constexpr uint32_t lds_vectors(uint32_t rows, uint32_t G) {
  return rows * G + (rows * G) / 16;
}

template <int V>
struct Vec;
template <>
struct Vec<4> {
  __device__ static void get(const uint32_t* p, int32_t (&x)[4]) {
    const uint4 t = *reinterpret_cast<const uint4*>(p);
    x[0] = t.x; x[1] = t.y; x[2] = t.z; x[3] = t.w;
  }
  __device__ static void put(uint32_t* p, const int32_t (&x)[4]) {
    *reinterpret_cast<uint4*>(p) = make_uint4(x[0], x[1], x[2], x[3]);
  }
};
template <>
struct Vec<2> {
  __device__ static void get(const uint32_t* p, int32_t (&x)[2]) {
    const uint2 t = *reinterpret_cast<const uint2*>(p);
    x[0] = t.x; x[1] = t.y;
  }
  __device__ static void put(uint32_t* p, const int32_t (&x)[2]) {
    *reinterpret_cast<uint2*>(p) = make_uint2(x[0], x[1]);
  }
};
template <>
struct Vec<1> {
  __device__ static void get(const uint32_t* p, int32_t (&x)[1]) { x[0] = (int32_t)p[0]; }
  __device__ static void put(uint32_t* p, const int32_t (&x)[1]) { p[0] = (uint32_t)x[0]; }
};

// Item I/O on the LDS tile: 2^B positions base + c*H of lane group g.
template <int B, int V, int G, uint32_t H>
__device__ __forceinline__ void lds_item_get(const uint32_t* lds, uint32_t base, uint32_t g,
                                             int32_t (&x)[1 << B][V]) {
  const uint32_t* p = lds + phys(base * G + g) * V;
#pragma unroll
  for (int c = 0; c < (1 << B); ++c) {
    constexpr uint32_t step = H * G;
    const uint32_t off = c * step + (c * step) / 16;
    Vec<V>::get(p + off * V, x[c]);
  }
}
template <int B, int V, int G, uint32_t H>
__device__ __forceinline__ void lds_item_put(uint32_t* lds, uint32_t base, uint32_t g,
                                             const int32_t (&x)[1 << B][V]) {
  uint32_t* p = lds + phys(base * G + g) * V;
#pragma unroll
  for (int c = 0; c < (1 << B); ++c) {
    constexpr uint32_t step = H * G;
    const uint32_t off = c * step + (c * step) / 16;
    Vec<V>::put(p + off * V, x[c]);
  }
}

// ---------------------------------------------------------------- twiddles
// A twiddle source yields w = omega_(2^lg)^j (j < 2^(lg-1)) for the forward
// root, or for the inverse root possibly as its negative (NEG): the
// butterflies then swap their +/- outputs, which costs nothing.
//
// TwGlobal: the 3^e and 3^-e tables in global memory (any size).
// TwLds<L>: tab[u] = omega_(2^L)^u, u <= 2^(L-1), in LDS; omega_(2^lg)^j =
//   tab[j 2^(L-lg)], and since omega_(2^L)^(2^(L-1)) = -1 the inverse is
//   omega^-u = -tab[2^(L-1) - u].
struct TwGlobal {
  const uint32_t* fwd;
  const uint32_t* inv;
  static constexpr bool NEG = false;
  __device__ __forceinline__ uint32_t get(bool inverse, uint32_t j, int lg) const {
    return gptr(inverse ? inv : fwd)[j << (16 - lg)];
  }
};

// TwLds<L, LO, TOP>: per-stage tables in LDS.  For LO <= lg <= TOP the table
// of stage lg holds omega_(2^lg)^j for j <= 2^(lg-1), contiguous in j, so the
// items of a pass (consecutive j) read consecutive words; the inverse root is
// omega^-j = -omega^(2^(lg-1) - j), read mirrored with NEG.  Stages above TOP
// read the table of stage L (omega_(2^L)^u, u <= 2^(L-1)) at stride
// 2^(L-lg).  Stages below LO are never looked up (the first pass of a
// transform uses compile-time roots).
template <int L, int LO, int TOP>
struct TwLds {
  const uint32_t* tab;
  static constexpr bool NEG = true;
  // word offset of the table of stage lg (LO <= lg <= TOP), then stage L
  __host__ __device__ static constexpr uint32_t off(int lg) {
    uint32_t o = 0;
    for (int g = LO; g < lg; ++g) o += (1u << (g - 1)) + 1;
    return o;
  }
  __host__ __device__ static constexpr uint32_t words() {
    return off(TOP + 1) + (TOP < L ? (1u << (L - 1)) + 1 : 0);
  }
  __device__ __forceinline__ uint32_t get(bool inverse, uint32_t j, int lg) const {
    if (lg <= TOP) return tab[off(lg) + (inverse ? (1u << (lg - 1)) - j : j)];
    const uint32_t u = j << (L - lg);
    return tab[off(TOP + 1) + (inverse ? (1u << (L - 1)) - u : u)];
  }
  // fills the tables from the context's stage tables (kStageTwBase after
  // tw[e] = 3^e): omega_(2^lg)^j = 3^(j 2^(16-lg))
  __device__ __forceinline__ void fill(uint32_t* t, const uint32_t* __restrict__ tw) const {
    const uint32_t* st = tw + kStageTwBase;
    for (int lg = LO; lg <= TOP; ++lg)
      for (uint32_t j = threadIdx.x; j <= (1u << (lg - 1)); j += blockDim.x) t[off(lg) + j] = gptr(st)[stage_tw_offset(lg) + j];
    if (TOP < L)
      for (uint32_t u = threadIdx.x; u <= (1u << (L - 1)); u += blockDim.x) t[off(TOP + 1) + u] = gptr(st)[stage_tw_offset(L) + u];
  }
  // the same from tw itself (strided reads): for a kernel at the edge of its
  // register budget, where the other form's addressing costs a spill
  __device__ __forceinline__ void fill_strided(uint32_t* t, const uint32_t* __restrict__ tw) const {
    for (int lg = LO; lg <= TOP; ++lg)
      for (uint32_t j = threadIdx.x; j <= (1u << (lg - 1)); j += blockDim.x) t[off(lg) + j] = gptr(tw)[j << (16 - lg)];
    if (TOP < L)
      for (uint32_t u = threadIdx.x; u <= (1u << (L - 1)); u += blockDim.x) t[off(TOP + 1) + u] = gptr(tw)[u << (16 - L)];
  }
};

// ---------------------------------------------------------------- butterflies
// DIT stages S0 + I0 .. S0 + B - 1 of an item (stages below I0 already
// applied by its loader).
template <int B, int V, int S0, bool INV, int I0 = 0, class TW>
__device__ __forceinline__ void dit_stages(int32_t (&x)[1 << B][V], uint32_t jp, const TW& tws) {
  static_assert(I0 >= 0 && I0 <= B, "stages to skip");
#pragma unroll
  for (int i = I0; i < B; ++i) {
    const int lg = S0 + i + 1;
#pragma unroll
    for (int cc = 0; cc < (1 << i); ++cc) {
      // twiddle omega_(2^lg)^(jp + cc 2^S0)
      uint32_t w = 1;
      bool triv = false, neg = false;
      if constexpr (S0 == 0) {
        triv = cc == 0;
        w = small_root<INV>(lg, cc);
      } else {
        w = tws.get(INV, jp + ((uint32_t)cc << S0), lg);
        neg = INV && TW::NEG;
      }
#pragma unroll
      for (int c0 = 0; c0 < (1 << B); c0 += 2 << i) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int32_t a = x[c0 + cc][v];
          const int32_t t = triv ? x[c0 + cc + (1 << i)][v] : mulw(x[c0 + cc + (1 << i)][v], w);
          x[c0 + cc][v] = neg ? a - t : a + t;
          x[c0 + cc + (1 << i)][v] = neg ? a + t : a - t;
        }
      }
    }
  }
}

// DIF stages with spans 2^(S1-1) down to 2^(S1-B), S1 = top stage index + 1.
template <int B, int V, int S1, bool INV, class TW>
__device__ __forceinline__ void dif_stages(int32_t (&x)[1 << B][V], uint32_t jp, const TW& tws) {
  constexpr int S0 = S1 - B;    // log2 of the item stride
#pragma unroll
  for (int i = B - 1; i >= 0; --i) {
    const int lg = S0 + i + 1;  // pairs at distance 2^(S0+i), block 2^lg
#pragma unroll
    for (int cc = 0; cc < (1 << i); ++cc) {
      uint32_t w = 1;
      bool triv = false, neg = false;
      if constexpr (S0 == 0) {
        triv = cc == 0;
        w = small_root<INV>(lg, cc);
      } else {
        w = tws.get(INV, jp + ((uint32_t)cc << S0), lg);
        neg = INV && TW::NEG;
      }
#pragma unroll
      for (int c0 = 0; c0 < (1 << B); c0 += 2 << i) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const int32_t a = x[c0 + cc][v], b = x[c0 + cc + (1 << i)][v];
          x[c0 + cc][v] = a + b;
          x[c0 + cc + (1 << i)][v] = triv ? a - b : mulw(neg ? b - a : a - b, w);
        }
      }
    }
  }
}

// ---------------------------------------------------------------- plans
// An L-stage transform with radix bound BM takes NP = ceil(L/BM) passes with
// radices as equal as possible.  DIT passes run bottom-up (pass 0 has stride
// 1) and put the larger radices first; DIF passes run top-down and put them
// last.  Either way the stride-1 pass gets the largest radix, which keeps the
// padded layout conflict-free there when that radix is 16 or more (or
// H*G >= 16); a radix-8 stride-1 pass over one lane group shares banks
// two-way.
__host__ __device__ constexpr int plan_np(int L, int BM) { return L == 0 ? 0 : (L + BM - 1) / BM; }
__host__ __device__ constexpr int plan_b(int L, int BM, int p) {
  return L / plan_np(L, BM) + (p < L % plan_np(L, BM) ? 1 : 0);
}
// DIT pass p covers stages [dit_s0, dit_s0 + B).
__host__ __device__ constexpr int dit_s0(int L, int BM, int p) {
  int s = 0;
  for (int q = 0; q < p; ++q) s += plan_b(L, BM, q);
  return s;
}
// DIF pass p has radix plan_b(L, BM, NP-1-p) and covers stages [top - B, top).
__host__ __device__ constexpr int dif_top(int L, int BM, int p) {
  int t = L;
  for (int q = 0; q < p; ++q) t -= plan_b(L, BM, plan_np(L, BM) - 1 - q);
  return t;
}

// Loaders / storers are objects with a member template
//   item<B, H>(base, g, x)  that moves the 2^B positions base + c*H of lane
// group g between their home (global memory or the LDS tile) and registers.
// A first-pass loader may declare kSkip: the number of leading DIT stages
// its items arrive with already applied.
template <class T, class = void>
struct loader_skip {
  static constexpr int value = 0;
};
template <class T>
struct loader_skip<T, std::void_t<decltype(T::kSkip)>> {
  static constexpr int value = T::kSkip;
};

template <int L, int BM, int P, int V, int G, bool INV, class TW, class Ld, class St>
__device__ __forceinline__ void dit_pass(const TW& tw, Ld& ld, St& st) {
  constexpr int B = plan_b(L, BM, P);
  constexpr int S0 = dit_s0(L, BM, P);
  constexpr int I0 = P == 0 ? loader_skip<Ld>::value : 0;
  constexpr uint32_t H = 1u << S0;
  constexpr uint32_t ITEMS = (1u << (L - B)) * G;
  for (uint32_t q = threadIdx.x; q < ITEMS; q += blockDim.x) {
    const uint32_t g = q % G, it = q / G;
    const uint32_t jp = it % H, blk = it / H;
    const uint32_t base = blk * (H << B) + jp;
    int32_t x[1 << B][V];
    ld.template item<B, H>(base, g, x);
    dit_stages<B, V, S0, INV, I0>(x, jp, tw);
    st.template item<B, H>(base, g, x);
  }
}

template <int L, int BM, int P, int V, int G, bool INV, class TW, class Ld, class St>
__device__ __forceinline__ void dif_pass(const TW& tw, Ld& ld, St& st) {
  constexpr int B = plan_b(L, BM, plan_np(L, BM) - 1 - P);
  constexpr int TOP = dif_top(L, BM, P);
  constexpr int S0 = TOP - B;
  constexpr uint32_t H = 1u << S0;
  constexpr uint32_t ITEMS = (1u << (L - B)) * G;
  for (uint32_t q = threadIdx.x; q < ITEMS; q += blockDim.x) {
    const uint32_t g = q % G, it = q / G;
    const uint32_t jp = it % H, blk = it / H;
    const uint32_t base = blk * (H << B) + jp;
    int32_t x[1 << B][V];
    ld.template item<B, H>(base, g, x);
    dif_stages<B, V, TOP, INV>(x, jp, tw);
    st.template item<B, H>(base, g, x);
  }
}

// Whole transforms: pass 0 uses (first-loader, mid-storer) ... the last pass
// (mid-loader, last-storer); a single-pass transform uses (first, last).
// A barrier follows every pass.
template <int L, int BM, int V, int G, bool INV, int P = 0, class TW, class L0, class LM, class SM, class SL>
__device__ __forceinline__ void dit(const TW& tw, L0& l0, LM& lm, SM& sm, SL& sl) {
  constexpr int NP = plan_np(L, BM);
  if constexpr (P < NP) {
    if constexpr (P == 0 && NP == 1) dit_pass<L, BM, P, V, G, INV>(tw, l0, sl);
    else if constexpr (P == 0) dit_pass<L, BM, P, V, G, INV>(tw, l0, sm);
    else if constexpr (P == NP - 1) dit_pass<L, BM, P, V, G, INV>(tw, lm, sl);
    else dit_pass<L, BM, P, V, G, INV>(tw, lm, sm);
    __syncthreads();
    dit<L, BM, V, G, INV, P + 1>(tw, l0, lm, sm, sl);
  }
}

template <int L, int BM, int V, int G, bool INV, int P = 0, class TW, class L0, class LM, class SM, class SL>
__device__ __forceinline__ void dif(const TW& tw, L0& l0, LM& lm, SM& sm, SL& sl) {
  constexpr int NP = plan_np(L, BM);
  if constexpr (P < NP) {
    if constexpr (P == 0 && NP == 1) dif_pass<L, BM, P, V, G, INV>(tw, l0, sl);
    else if constexpr (P == 0) dif_pass<L, BM, P, V, G, INV>(tw, l0, sm);
    else if constexpr (P == NP - 1) dif_pass<L, BM, P, V, G, INV>(tw, lm, sl);
    else dif_pass<L, BM, P, V, G, INV>(tw, lm, sm);
    __syncthreads();
    dif<L, BM, V, G, INV, P + 1>(tw, l0, lm, sm, sl);
  }
}

// Passes [P, Q) of a DIT transform (pass 0 reads through l0, the others
// through lm; all store through sm), a barrier after each.
template <int L, int BM, int V, int G, bool INV, int P, int Q, class TW, class L0, class LM, class SM>
__device__ __forceinline__ void dit_passes(const TW& tw, L0& l0, LM& lm, SM& sm) {
  if constexpr (P < Q) {
    if constexpr (P == 0) dit_pass<L, BM, 0, V, G, INV>(tw, l0, sm);
    else dit_pass<L, BM, P, V, G, INV>(tw, lm, sm);
    __syncthreads();
    dit_passes<L, BM, V, G, INV, P + 1, Q>(tw, l0, lm, sm);
  }
}

// Passes [P, Q) of a DIF transform through lm and sm, a barrier after each.
template <int L, int BM, int V, int G, bool INV, int P, int Q, class TW, class LM, class SM>
__device__ __forceinline__ void dif_passes(const TW& tw, LM& lm, SM& sm) {
  if constexpr (P < Q) {
    dif_pass<L, BM, P, V, G, INV>(tw, lm, sm);
    __syncthreads();
    dif_passes<L, BM, V, G, INV, P + 1, Q>(tw, lm, sm);
  }
}

// The last pass of one transform and the first pass of the next, over the
// same 2^L points, in one pass: a DIT transform ends with its top stages and
// a DIF transform starts with them (A_DIT), a DIF transform ends with its
// bottom stages and a DIT transform starts with them (!A_DIT); either way the
// two passes group the same positions, so a thread goes on with its item in
// registers, mid(base, g, x) in between, and the data crosses LDS once.
template <int L, int BM, int V, int G, bool A_DIT, bool A_INV, bool B_INV, class TW, class LM, class Mid, class SM>
__device__ __forceinline__ void seam_pass(const TW& tw, LM& lm, Mid& mid, SM& sm) {
  constexpr int NP = plan_np(L, BM);
  constexpr int B = A_DIT ? plan_b(L, BM, NP - 1) : plan_b(L, BM, 0);
  constexpr int S0 = A_DIT ? L - B : 0;
  static_assert(!A_DIT || dit_s0(L, BM, NP - 1) == S0, "a DIT transform ends with its top stages");
  static_assert(A_DIT || dif_top(L, BM, NP - 1) == B, "a DIF transform ends with its bottom stages");
  constexpr uint32_t H = 1u << S0;
  constexpr uint32_t ITEMS = (1u << (L - B)) * G;
  for (uint32_t q = threadIdx.x; q < ITEMS; q += blockDim.x) {
    const uint32_t g = q % G, it = q / G;
    const uint32_t jp = it % H, blk = it / H;
    const uint32_t base = blk * (H << B) + jp;
    int32_t x[1 << B][V];
    lm.template item<B, H>(base, g, x);
    if constexpr (A_DIT) dit_stages<B, V, S0, A_INV>(x, jp, tw);
    else dif_stages<B, V, S0 + B, A_INV>(x, jp, tw);
    mid.template item<B, H>(base, g, x);
    if constexpr (A_DIT) dif_stages<B, V, S0 + B, B_INV>(x, jp, tw);
    else dit_stages<B, V, S0, B_INV>(x, jp, tw);
    sm.template item<B, H>(base, g, x);
  }
}

// ---------------------------------------------------------------- pipeline
// Persistent kernels overlap the global reads of the next tile with the last
// pass of the current one: pass 0's inputs are read into registers ahead of
// time (raw<B>), completed when pass 0 runs (finish<B>: twist, weights), and
// the stores of the last pass drain while the next tile starts.  This needs
// every thread to own the same whole number C0 of pass-0 items.
template <int L, int BM, int G, int NT>
__host__ __device__ constexpr int pass0_per_thread() {
  return (((1u << (L - plan_b(L, BM, 0))) * G) % NT == 0) ? (int)(((1u << (L - plan_b(L, BM, 0))) * G) / NT) : 0;
}
// Pass-0 items of a thread when the threads outnumber them or do not split
// them evenly: ceil(items / NT) slots, of which the last may be empty.
template <int L, int BM, int G, int NT>
__host__ __device__ constexpr int pass0_slots() {
  return (int)(((1u << (L - plan_b(L, BM, 0))) * G + NT - 1) / NT);
}
template <int L, int BM, int G>
__host__ __device__ constexpr uint32_t pass0_items() {
  return (1u << (L - plan_b(L, BM, 0))) * G;
}

// Reads the per-position values of this thread's pass-0 items that every
// tile of a job shares (loader member consts<B>).
template <int L, int BM, int V, int G, int NT, int C0, class Ld>
__device__ __forceinline__ void consts0(Ld& ld, uint32_t (&aux)[C0][1 << plan_b(L, BM, 0)],
                                       uint32_t (&aux2)[C0][1 << plan_b(L, BM, 0)]) {
  constexpr int B = plan_b(L, BM, 0);
#pragma unroll
  for (int c = 0; c < C0; ++c) {
    const uint32_t q = threadIdx.x + (uint32_t)c * NT;
    if (q >= pass0_items<L, BM, G>()) continue;
    ld.template consts<B>((q / G) << B, aux[c], aux2[c]);
  }
}

// Issues the reads of this thread's pass-0 items (positions base + c,
// stride 1) of the loader's tile into x (loader member raw<B>), consuming
// none of them.
template <int L, int BM, int V, int G, int NT, int C0, class Ld>
__device__ __forceinline__ void prefetch0(Ld& ld, int32_t (&x)[C0][1 << plan_b(L, BM, 0)][V],
                                         uint32_t (&aux)[C0][1 << plan_b(L, BM, 0)],
                                         uint32_t (&aux2)[C0][1 << plan_b(L, BM, 0)]) {
  constexpr int B = plan_b(L, BM, 0);
#pragma unroll
  for (int c = 0; c < C0; ++c) {
    const uint32_t q = threadIdx.x + (uint32_t)c * NT;
    if (q >= pass0_items<L, BM, G>()) continue;
    const uint32_t g = q % G, it = q / G;
    ld.template raw<B>(it << B, g, x[c], aux[c], aux2[c]);
  }
}

// Pass 0 of a DIT transform from prefetched registers.
template <int L, int BM, int V, int G, int NT, int C0, bool INV, class TW, class Ld, class St>
__device__ __forceinline__ void dit_pass0_regs(const TW& tw, Ld& ld, int32_t (&pre)[C0][1 << plan_b(L, BM, 0)][V],
                                               uint32_t (&aux)[C0][1 << plan_b(L, BM, 0)],
                                               uint32_t (&aux2)[C0][1 << plan_b(L, BM, 0)], St& st) {
  constexpr int B = plan_b(L, BM, 0);
#pragma unroll
  for (int c = 0; c < C0; ++c) {
    const uint32_t q = threadIdx.x + (uint32_t)c * NT;
    if (q >= pass0_items<L, BM, G>()) continue;
    const uint32_t g = q % G, it = q / G;
    const uint32_t base = it << B;
    int32_t x[1 << B][V];
#pragma unroll
    for (int r = 0; r < (1 << B); ++r)
#pragma unroll
      for (int v = 0; v < V; ++v) x[r][v] = pre[c][r][v];
    ld.template finish<B>(base, g, x, aux[c], aux2[c]);
    dit_stages<B, V, 0, INV>(x, 0, tw);
    st.template item<B, 1>(base, g, x);
  }
}

// Passes P.. of a DIT transform (pass P reads through lm); hook() runs right
// before the last pass, and no barrier follows it.
template <int L, int BM, int V, int G, bool INV, int P, class TW, class LM, class SM, class SL, class Hook>
__device__ __forceinline__ void dit_from(const TW& tw, LM& lm, SM& sm, SL& sl, Hook& hook) {
  constexpr int NP = plan_np(L, BM);
  if constexpr (P < NP) {
    if constexpr (P == NP - 1) {
      hook();
      dit_pass<L, BM, P, V, G, INV>(tw, lm, sl);
    } else {
      dit_pass<L, BM, P, V, G, INV>(tw, lm, sm);
      __syncthreads();
      dit_from<L, BM, V, G, INV, P + 1>(tw, lm, sm, sl, hook);
    }
  }
}

// A whole DIT transform like dit<>, with hook() right before the last pass
// and no barrier after it.
template <int L, int BM, int V, int G, bool INV, class TW, class L0, class LM, class SM, class SL, class Hook>
__device__ __forceinline__ void dit_hooked(const TW& tw, L0& l0, LM& lm, SM& sm, SL& sl, Hook& hook) {
  if constexpr (plan_np(L, BM) == 1) {
    hook();
    dit_pass<L, BM, 0, V, G, INV>(tw, l0, sl);
  } else {
    dit_pass<L, BM, 0, V, G, INV>(tw, l0, sm);
    __syncthreads();
    dit_from<L, BM, V, G, INV, 1>(tw, lm, sm, sl, hook);
  }
}

struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};

}  // namespace ct
}  // namespace fntrs
