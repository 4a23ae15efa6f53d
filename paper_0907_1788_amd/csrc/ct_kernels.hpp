// Encoder and decoder kernels on compile-time transform plans (ctfnt.hpp).
// One workgroup owns a tile of T lanes of one codeword block; every
// transform of that block runs on chip, so each block crosses HBM once in
// each direction.
#pragma once
#include "codec_args.hpp"
#include "ctfnt.hpp"

#include <type_traits>

namespace fntrs {
namespace ct {

// Radix bound of the pass plan for a size-2^L transform on G lane groups of V
// lanes: aim for kThreads items per pass (items = G 2^(L-B)), radix 8 at
// least, the register budget of V lanes at most, and no more passes than
// needed while a pass keeps at least half the threads busy -- all of them in
// a 1024-thread workgroup, which has its CU to itself: a half-idle pass would
// leave the CU 8 waves for a third of the butterflies.
__host__ __device__ constexpr int geo_bm(int L, int G, int V, int NT) {
  int lg = 0, lt = 0;
  while ((1 << lg) < G) ++lg;
  while ((1 << lt) < NT) ++lt;
  // radix 2^5 at most: a first pass of trivial butterflies grows a value by
  // 2^B and the multiplier takes 24-bit operands
  const int bmax = V == 4 ? 4 : 5;
  int b = L + lg - lt;
  if (b < 3) b = 3;
  if (b > bmax) b = bmax;
  if (b > L) b = L;
  if (b < 1) b = 1;
  // a larger radix that saves a pass while items >= kThreads/2 (kThreads
  // with 1024 threads)
  const int busy = NT >= 1024 ? NT : NT / 2;
  for (int c = b + 1; c <= bmax && c <= L; ++c)
    if ((L + c - 1) / c < (L + b - 1) / b && (G << (L - c)) >= busy) return c;
  return b;
}

// Tile geometry: T lanes per tile, V lanes per thread (VV, or 4 when the
// tile allows), G = T/V lane groups, NT threads, radix bound BM, LDS bytes of
// the padded tile.
template <int L, int T_, int NT_, int VV = 0>
struct Geo {
  static constexpr int T = T_;
  static constexpr int NT = NT_;
  static constexpr int V = VV ? VV : (T >= 4 ? 4 : T);   // lanes per thread (vector width)
  static_assert(T % V == 0, "the tile must hold whole vectors");
  static constexpr int G = T / V;
  static constexpr int BM = geo_bm(L, G, V, NT);
  static constexpr uint32_t TILE_BYTES = lds_vectors(1u << L, G) * V * 4;
  // LDS twiddle tables (TwLds): stages from the second pass up; all stages in
  // per-stage tables when they fit, else the top two stages share the
  // stage-L table; none when even that does not fit (global tables then)
  // (the decoder's size-2^(L-1) transforms start with their own first pass)
  static constexpr int LO = (L > 1 && plan_b(L - 1, BM, 0) < plan_b(L, BM, 0) ? plan_b(L - 1, BM, 0)
                                                                                : plan_b(L, BM, 0)) + 1;
  // Stages up to TOP get their own tables, the stages above read the stage-L
  // table at a stride.  TOP is the highest stage whose tables still let as
  // many workgroups share a CU's LDS as the smallest tables would (strided
  // reads of the small low-stage tables would conflict on LDS banks, so
  // those keep their own tables whenever that costs no occupancy).
  static constexpr uint32_t kLds = 163840;
  static constexpr uint32_t words_at(int top) {
    return TwLds<L, LO, L>::off(top + 1) + (top < L ? (1u << (L - 1)) + 1 : 0);
  }
  static constexpr uint32_t wgs(int top) { return kLds / (TILE_BYTES + words_at(top) * 4); }
  static constexpr int pick_top() {
    int t = L;
    while (t >= LO && wgs(t) < wgs(LO - 1)) --t;
    return t < LO - 1 ? LO - 1 : t;
  }
  static constexpr int TOP = LO <= L ? pick_top() : L;
  static constexpr uint32_t WORDS = TwLds<L, LO, TOP>::words();
  static constexpr bool TW_LDS = LO <= L && TILE_BYTES + WORDS * 4 <= kLds;
  static constexpr uint32_t LDS_BYTES = TILE_BYTES + (TW_LDS ? WORDS * 4 : 0);
  using TwType = typename std::conditional<TW_LDS, TwLds<L, LO, TOP>, TwGlobal>::type;
};

// STRIDED: fill the LDS tables from tw itself (TwLds::fill_strided).
template <bool STRIDED = false, int L, int LO, int TOP>
__device__ __forceinline__ TwLds<L, LO, TOP> make_tw(const TwLds<L, LO, TOP>*, uint32_t* lds_tab, const uint32_t* tw,
                                                      const uint32_t*) {
  TwLds<L, LO, TOP> t{lds_tab};
  if constexpr (STRIDED) t.fill_strided(lds_tab, tw);
  else t.fill(lds_tab, tw);
  return t;
}
template <bool STRIDED = false>
__device__ __forceinline__ TwGlobal make_tw(const TwGlobal*, uint32_t*, const uint32_t* tw, const uint32_t* twi) {
  return TwGlobal{tw, twi};
}

// ---------------------------------------------------------------- LDS movers
template <int V, int G>
struct LdsLoad {
  const uint32_t* lds;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    lds_item_get<B, V, G, H>(lds, base, g, x);
  }
};

template <int V, int G, bool FOLD>
struct LdsStore {
  uint32_t* lds;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    if constexpr (FOLD) {
#pragma unroll
      for (int c = 0; c < (1 << B); ++c)
#pragma unroll
        for (int v = 0; v < V; ++v) x[c][v] = fold1(x[c][v]);
    }
    lds_item_put<B, V, G, H>(lds, base, g, x);
  }
};

// 64-bit row address helper: rows are `ld` elements apart.
__device__ __forceinline__ const uint32_t* row_ptr(const uint32_t* p, uint64_t row, uint64_t ld) {
  return p + row * ld;
}

// One row of V lanes as int32, whole (one access) or part (ragged tail).
template <int V, bool WHOLE>
__device__ __forceinline__ void load_lanes(const uint32_t* p, uint32_t lane, uint32_t lanes, int32_t (&x)[V]) {
  uint32_t u[V];
  if constexpr (WHOLE) gload_whole<V>(p, u);
  else gload_part<V>(p, lane, lanes, u);
#pragma unroll
  for (int v = 0; v < V; ++v) x[v] = (int32_t)u[v];
}

template <int V, bool WHOLE>
__device__ __forceinline__ void store_lanes(uint32_t* p, uint32_t lane, uint32_t lanes, const int32_t (&x)[V]) {
  uint32_t u[V];
#pragma unroll
  for (int v = 0; v < V; ++v) u[v] = canon(x[v]);
  if constexpr (WHOLE) gstore_whole<V>(p, u);
  else gstore_part<V>(p, lane, lanes, u);
}

// ---------------------------------------------------------------- encoder
// First DIT pass of the encoder: position pos holds source row bitrev(pos),
// twisted by r_n^(t j) (coset t); rows j >= k are zero padding.  raw issues
// all reads of an item -- the rows and their twist factors -- before finish
// consumes any of them (twist, zero the padding).
template <int L, int V>
struct EncLoad {
  const uint32_t* src;
  const uint32_t* tw;
  uint64_t ld;
  uint32_t k, n, t, lane0, lanes;
  int sh;
  bool vec;
  template <int B, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t jb, uint32_t g, int32_t (&x)[1 << B][V], uint32_t (&wt)[1 << B]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t j = jb | (bitrev((uint32_t)c, B) << (L - B));
      wt[c] = gptr(tw)[((t * j) & (n - 1)) << sh];   // tw[0] = 1 for coset 0
      // no branch: a padding row reads row k-1 (finish zeroes it), which
      // keeps the reads of an item one straight sequence
      const uint32_t jr = j < k ? j : k - 1;
      load_lanes<V, WHOLE>(row_ptr(src, jr, ld) + g * V, lane0 + g * V, lanes, x[c]);
    }
  }
  template <int B>
  __device__ __forceinline__ void raw(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V], uint32_t (&wt)[1 << B],
                                      uint32_t (&)[1 << B]) {
    const uint32_t jb = bitrev(base, L);
    if (whole_vector<V>(lane0 + g * V, lanes, vec)) rows<B, true>(jb, g, x, wt);
    else rows<B, false>(jb, g, x, wt);
  }
  template <int B>
  __device__ __forceinline__ void finish(uint32_t base, uint32_t, int32_t (&x)[1 << B][V], const uint32_t (&wt)[1 << B],
                                         const uint32_t (&)[1 << B]) {
    const uint32_t jb = bitrev(base, L);
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t j = jb | (bitrev((uint32_t)c, B) << (L - B));
#pragma unroll
      for (int v = 0; v < V; ++v) x[c][v] = j < k ? (t ? mulw(x[c][v], wt[c]) : x[c][v]) : 0;
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    static_assert(H == 1, "the first DIT pass has stride 1");
    uint32_t aux[1 << B], aux2[1 << B];
    raw<B>(base, g, x, aux, aux2);
    finish<B>(base, g, x, aux, aux2);
  }
  // the twist factors of coset 1 of two (n = 2K) for the positions of the
  // item at base, from the transform's own twiddle source: r_n^j =
  // omega_K^(j/2), times r_n for odd j (the item's positions share j's parity)
  template <int B, class TW>
  __device__ __forceinline__ void twists_half(uint32_t base, uint32_t (&wt)[1 << B], const TW& tws,
                                              uint32_t rn) const {
    const uint32_t jb = bitrev(base, L);
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t j = jb | (bitrev((uint32_t)c, B) << (L - B));
      const uint32_t w = tws.get(false, j >> 1, L);
      wt[c] = (jb & 1u) ? canon(mulw((int32_t)w, rn)) : w;
    }
  }
  // the twist factors of coset t for the positions of the item at base
  template <int B>
  __device__ __forceinline__ void twists(uint32_t base, uint32_t (&wt)[1 << B]) const {
    const uint32_t jb = bitrev(base, L);
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t j = jb | (bitrev((uint32_t)c, B) << (L - B));
      wt[c] = gptr(tw)[((t * j) & (n - 1)) << sh];
    }
  }
};

// Last DIT pass of the encoder: output m of coset t is row t + cosets*m.
template <int V>
struct EncStore {
  uint32_t* dst;
  uint64_t ld;
  uint32_t t, cosets, lane0, lanes;
  bool vec;
  uint32_t rows_out;   // rows at or beyond are not written (0: none skipped)
  template <int B, uint32_t H, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint64_t row = t + (uint64_t)cosets * (base + c * H);
      if (rows_out && row >= rows_out) continue;
      store_lanes<V, WHOLE>(dst + row * ld + g * V, lane0 + g * V, lanes, x[c]);
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    if (whole_vector<V>(lane0 + g * V, lanes, vec)) rows<B, H, true>(base, g, x);
    else rows<B, H, false>(base, g, x);
  }
};

// Encoder, Sec. II-B: e_i = s(r_n^i).  Output row t + (n/K) m is output m of
// FNT_K of (s_j r_n^(t j))_j (r_n^(n/K) = r_K), one work item per
// (coset t, lane tile, block), coset fastest.
template <int LK, int TT, int NT, int VV, class TW>
__device__ __forceinline__ void enc_item(const EncodeArgs& a, uint32_t item, uint32_t* lds, const TW& tws) {
  using Gm = Geo<LK, TT, NT, VV>;
  constexpr int V = Gm::V, G = Gm::G, T = Gm::T;
  const uint32_t t = item % a.cosets;
  item /= a.cosets;
  const uint32_t tile = item % a.tiles;
  const uint64_t blk = item / a.tiles;
  const uint32_t lane0 = tile * T;
  EncLoad<LK, V> l0{a.src + blk * a.stride_src + lane0, a.tw, a.ld_src, a.k, a.n, t, lane0, a.lanes,
                    16 - a.logn, a.vec != 0};
  LdsLoad<V, G> lm{lds};
  LdsStore<V, G, false> sm{lds};
  EncStore<V> sl{a.dst + blk * a.stride_dst + lane0, a.ld_dst, t, a.cosets, lane0, a.lanes, a.vec != 0, a.rows_out};
  dit<LK, Gm::BM, V, G, false>(tws, l0, lm, sm, sl);
}

// Encoder with every coset of a lane tile in one workgroup: the tile's
// source rows are read once into registers (pass-0 items, C0 slots per
// thread), and each coset's first pass twists them there; the stores of one
// coset drain while the next computes.  Work item = (lane tile, block).
template <int LK, int TT, int NT, int VV>
struct EncCosRegs {
  using Gm = Geo<LK, TT, NT, VV>;
  static constexpr int V = Gm::V, B0 = plan_b(LK, Gm::BM, 0), C0 = pass0_slots<LK, Gm::BM, Gm::G, NT>();
  int32_t src[C0][1 << B0][V];
  uint32_t wt[C0][1 << B0], unused[C0][1 << B0];
};

// The loader of item `item` of job `a` (coset 0).
template <int LK, int TT, int NT, int VV>
__device__ __forceinline__ EncLoad<LK, Geo<LK, TT, NT, VV>::V> enc_cos_loader(const EncodeArgs& a, uint32_t item) {
  using Gm = Geo<LK, TT, NT, VV>;
  const uint32_t lane0 = (item % a.tiles) * Gm::T;
  const uint64_t blk = item / a.tiles;
  return {a.src + blk * a.stride_src + lane0, a.tw, a.ld_src, a.k, a.n, 0u, lane0, a.lanes, 16 - a.logn, a.vec != 0};
}

// Reads the source rows of item `item` into the registers (coset 0: no twist).
template <int LK, int TT, int NT, int VV>
__device__ __forceinline__ void enc_cos_prefetch(const EncodeArgs& a, uint32_t item, EncCosRegs<LK, TT, NT, VV>& r) {
  using Gm = Geo<LK, TT, NT, VV>;
  auto ld = enc_cos_loader<LK, TT, NT, VV>(a, item);
  prefetch0<LK, Gm::BM, Gm::V, Gm::G, NT, EncCosRegs<LK, TT, NT, VV>::C0>(ld, r.src, r.wt, r.unused);
}

// Every coset of item `item` from the rows in `r`; `last` runs once the last
// coset's first pass has consumed the rows in `r` (a persistent kernel reads
// the next item's rows there, and that read overlaps every later pass).
template <int LK, int TT, int NT, int VV, class TW, class Hook>
__device__ __forceinline__ void enc_cos_body(const EncodeArgs& a, uint32_t item, uint32_t* lds, const TW& tws,
                                             EncCosRegs<LK, TT, NT, VV>& r, Hook& last) {
  using Gm = Geo<LK, TT, NT, VV>;
  constexpr int V = Gm::V, G = Gm::G, T = Gm::T, BM = Gm::BM;
  constexpr int B0 = EncCosRegs<LK, TT, NT, VV>::B0, C0 = EncCosRegs<LK, TT, NT, VV>::C0;
  static_assert(plan_np(LK, BM) >= 2, "needs a first and a last pass");
  const uint32_t lane0 = (item % a.tiles) * T;
  const uint64_t blk = item / a.tiles;
  auto ld = enc_cos_loader<LK, TT, NT, VV>(a, item);
  const uint32_t rn = gptr(a.tw)[1u << (16 - a.logn)];     // r_n
  LdsLoad<V, G> lm{lds};
  LdsStore<V, G, false> sm{lds};
  NoHook none;
  for (uint32_t t = 0; t < a.cosets; ++t) {
    ld.t = t;
    if (t) {
#pragma unroll
      for (int c = 0; c < C0; ++c) {
        if (threadIdx.x + (uint32_t)c * NT >= pass0_items<LK, BM, G>()) continue;
        const uint32_t base = ((threadIdx.x + (uint32_t)c * NT) / G) << B0;
        // two cosets: the factors come from the twiddle table (LDS), so they
        // do not wait behind the previous coset's stores
        if (a.cosets == 2) ld.template twists_half<B0>(base, r.wt[c], tws, rn);
        else ld.template twists<B0>(base, r.wt[c]);
      }
    }
    dit_pass0_regs<LK, BM, V, G, NT, C0, false>(tws, ld, r.src, r.wt, r.unused, sm);
    __syncthreads();
    EncStore<V> sl{a.dst + blk * a.stride_dst + lane0, a.ld_dst, t, a.cosets, lane0, a.lanes, a.vec != 0,
                   a.rows_out};
    if (t + 1 == a.cosets) last();
    dit_from<LK, BM, V, G, false, 1>(tws, lm, sm, sl, none);
    __syncthreads();   // the next coset's (or item's) first pass overwrites the LDS tile
  }
}

template <int LK, int TT, int NT, int VV, class TW>
__device__ __forceinline__ void enc_cos_item(const EncodeArgs& a, uint32_t item, uint32_t* lds, const TW& tws) {
  EncCosRegs<LK, TT, NT, VV> r;
  enc_cos_prefetch<LK, TT, NT, VV>(a, item, r);
  NoHook none;
  enc_cos_body<LK, TT, NT, VV>(a, item, lds, tws, r, none);
}

template <int LK, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_enc_cos(EncodeArgs a) {
  using Gm = Geo<LK, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  // the kernel holds a tile's source across its cosets at the edge of its
  // register budget: the strided fill keeps it from spilling
  const TW tws = make_tw<true>((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  enc_cos_item<LK, TT, NT, VV>(a, xcd_remap(blockIdx.x, gridDim.x), lds, tws);
}

template <int LK, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_enc(EncodeArgs a) {
  using Gm = Geo<LK, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  enc_item<LK, TT, NT, VV>(a, xcd_remap(blockIdx.x, gridDim.x), lds, tws);
}

// Job of work item w: the last j with start[j] <= w (uniform per workgroup).
__device__ __forceinline__ uint32_t find_job(const uint32_t* start, uint32_t njobs, uint32_t w) {
  uint32_t lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (gptr(start)[mid] <= w) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Batched encoder: a persistent grid walks the work items of every job of
// one transform size; the LDS twiddle tables are filled once per workgroup.
template <int LK, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_enc_tab(JobTable<EncodeArgs> t, const uint32_t* tw, const uint32_t* twi) {
  using Gm = Geo<LK, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, tw, twi);
  for (uint32_t w = xcd_remap(blockIdx.x, gridDim.x); w < t.total; w += gridDim.x) {
    const uint32_t j = find_job(t.start, t.njobs, w);
    const EncodeArgs a = load_global(t.jobs + j);
    enc_item<LK, TT, NT, VV>(a, w - gptr(t.start)[j], lds, tws);
    __syncthreads();   // the next item overwrites the LDS tile
  }
}

// Batched all-cosets encoder: as k_enc_tab, but a work item is a (lane tile,
// block) whose every coset the workgroup computes from one load of the
// source rows (k_enc_cos).
// The next item's source rows are read into the registers as soon as the
// current item's last coset has consumed them (after its first pass), so
// their latency overlaps that coset's remaining passes and its stores.
template <int LK, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_enc_cos_tab(JobTable<EncodeArgs> t, const uint32_t* tw, const uint32_t* twi) {
  using Gm = Geo<LK, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, tw, twi);
  uint32_t w = xcd_remap(blockIdx.x, gridDim.x);
  if (w >= t.total) return;
  EncCosRegs<LK, TT, NT, VV> r;
  {
    const uint32_t j = find_job(t.start, t.njobs, w);
    enc_cos_prefetch<LK, TT, NT, VV>(load_global(t.jobs + j), w - gptr(t.start)[j], r);
  }
  for (; w < t.total; w += gridDim.x) {
    const uint32_t j = find_job(t.start, t.njobs, w);
    const EncodeArgs a = load_global(t.jobs + j);
    const uint32_t wn = w + gridDim.x;
    auto next = [&]() {
      if (wn < t.total) {
        const uint32_t jn = find_job(t.start, t.njobs, wn);
        enc_cos_prefetch<LK, TT, NT, VV>(load_global(t.jobs + jn), wn - gptr(t.start)[jn], r);
      }
    };
    enc_cos_body<LK, TT, NT, VV>(a, w - gptr(t.start)[j], lds, tws, r, next);
  }
}

// The job and local work item of global work item w: from the table, or the
// single job `one` when the table has none.
template <class Args>
__device__ __forceinline__ Args job_at(const JobTable<Args>& t, const Args& one, uint32_t w, uint32_t& local,
                                       uint32_t& job) {
  if (!t.jobs) {
    local = w;
    job = 0;
    return one;
  }
  const uint32_t j = find_job(t.start, t.njobs, w);
  local = w - gptr(t.start)[j];
  job = j;
  return load_global(t.jobs + j);
}

// ---------------------------------------------------------------- decoder
// First DIT pass of step 5: position pos holds u at index z = bitrev(pos):
// the received symbol v_z times the locator weight of z (0 if z is erased).
// consts reads the weights and rows of the positions (the same for every
// tile of a locator), raw issues the row reads of all positions and
// consumes nothing, finish multiplies and zeroes the erased positions.
template <int L, int V>
struct DecLoad {
  const uint32_t* recv;
  const uint32_t* wfull;
  const uint32_t* ridx;
  uint64_t ld;
  uint32_t lane0, lanes, row0;
  bool full, vec;
  const uint32_t* wrb;   // DecodeArgs::wrb
  template <int B>
  __device__ __forceinline__ void consts(uint32_t base, uint32_t (&wv)[1 << B], uint32_t (&rv)[1 << B]) {
    if (wrb) {   // uniform: the pairs of positions bitrev(base + c) lie together
#pragma unroll
      for (int c = 0; c < (1 << B); ++c) {
        const u32x2 q = *(const FNTRS_GLOBAL u32x2*)gptr(wrb + 2 * (base + c));
        wv[c] = q.x;
        rv[c] = q.x ? q.y : row0;
      }
      return;
    }
    const uint32_t zb = bitrev(base, L);
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t z = zb | (bitrev((uint32_t)c, B) << (L - B));
      const uint32_t w = gptr(wfull)[z];
      wv[c] = w;
      // an erased position reads a received row, which the tile reads
      // anyway (no extra HBM traffic); finish zeroes it
      rv[c] = w ? (full ? z : gptr(ridx)[z]) : row0;
    }
  }
  template <int B, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t g, int32_t (&x)[1 << B][V], const uint32_t (&wv)[1 << B],
                                       const uint32_t (&rv)[1 << B]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c)
      load_lanes<V, WHOLE>(row_ptr(recv, rv[c], ld) + g * V, lane0 + g * V, lanes, x[c]);
  }
  template <int B>
  __device__ __forceinline__ void raw(uint32_t, uint32_t g, int32_t (&x)[1 << B][V], uint32_t (&wv)[1 << B],
                                      uint32_t (&rv)[1 << B]) {
    if (whole_vector<V>(lane0 + g * V, lanes, vec)) rows<B, true>(g, x, wv, rv);
    else rows<B, false>(g, x, wv, rv);
  }
  template <int B>
  __device__ __forceinline__ void finish(uint32_t, uint32_t, int32_t (&x)[1 << B][V], const uint32_t (&wv)[1 << B],
                                         const uint32_t (&)[1 << B]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c)
#pragma unroll
      for (int v = 0; v < V; ++v) x[c][v] = wv[c] ? mulc((uint32_t)x[c][v], wv[c]) : 0;
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    static_assert(H == 1, "the first DIT pass has stride 1");
    uint32_t wv[1 << B], rv[1 << B];
    consts<B>(base, wv, rv);
    raw<B>(base, g, x, wv, rv);
    finish<B>(base, g, x, wv, rv);
  }
};

// Last pass of step 5: keep S_m = U_m for m < k (folded: the DIF transform
// that follows doubles ranges), zero for k <= m < M (the padding of the
// length-M product), positions >= M are never read.
template <int V, int G>
struct SeriesStore {
  uint32_t* lds;
  uint32_t k;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t m = base + c * H;
#pragma unroll
      for (int v = 0; v < V; ++v) x[c][v] = m < k ? fold1(x[c][v]) : 0;
    }
    // positions >= 2k are never read again; writing them is harmless
    lds_item_put<B, V, G, H>(lds, base, g, x);
  }
};

// Last DIF pass of step 6: multiply the transform of S (bit-reversed order)
// by the locator's FNT_2k(A mod x^k)/2k, stored in the same order.
template <int V, int G>
struct ProductStore {
  uint32_t* lds;
  const uint32_t* ahat_br;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t h = gptr(ahat_br)[base + c * H];
#pragma unroll
      for (int v = 0; v < V; ++v) x[c][v] = mulc(canon(x[c][v]), h);
    }
    lds_item_put<B, V, G, H>(lds, base, g, x);
  }
};

// The same two operations at the seams of the decoder's transforms, where
// the data stays in registers (seam_pass): the series mask of step 5, and the
// product with FNT_M(A mod x^k)/M in bit-reversed order.
template <int V>
struct SeriesMask {
  uint32_t k;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t, int32_t (&x)[1 << B][V]) const {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t m = base + c * H;
#pragma unroll
      for (int v = 0; v < V; ++v) x[c][v] = m < k ? fold1(x[c][v]) : 0;
    }
  }
};
template <int V>
struct AhatProduct {
  const uint32_t* ahat_br;
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t, int32_t (&x)[1 << B][V]) const {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t h = gptr(ahat_br)[base + c * H];
#pragma unroll
      for (int v = 0; v < V; ++v) x[c][v] = mulc(canon(x[c][v]), h);
    }
  }
};

// Last DIT pass of step 6: coefficients m < k are the recovered source rows.
template <int V>
struct SourceStore {
  uint32_t* dst;
  uint64_t ld;
  uint32_t k, lane0, lanes;
  bool vec;
  template <int B, uint32_t H, bool WHOLE>
  __device__ __forceinline__ void rows(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
#pragma unroll
    for (int c = 0; c < (1 << B); ++c) {
      const uint32_t m = base + c * H;
      if (m < k) store_lanes<V, WHOLE>(dst + (uint64_t)m * ld + g * V, lane0 + g * V, lanes, x[c]);
    }
  }
  template <int B, uint32_t H>
  __device__ __forceinline__ void item(uint32_t base, uint32_t g, int32_t (&x)[1 << B][V]) {
    if (whole_vector<V>(lane0 + g * V, lanes, vec)) rows<B, H, true>(base, g, x);
    else rows<B, H, false>(base, g, x);
  }
};

// Decoder, Sec. II-B steps 4-6, for n = 2^LN, k < n, and a product length
// M = 2^(LN-D) >= 2k (D in {0, 1}; any cyclic length >= 2k-1 makes the
// low product exact):
//   step 4+5: u_z = weight_z v_z (the locator folds -x_z^(-1)/A'(x_z) into
//             the weight), S_j = sum_z u_z r^(-j z) for j < k: inverse DIT
//             FNT_n, inputs read from global memory in bit-reversed order;
//   step 6:   P = (A S) mod x^k: DIF FNT_M of (S, 0) (natural in,
//             bit-reversed out), times FNT_M(A mod x^k)/M, inverse DIT FNT_M
//             (bit-reversed in, natural out); keep m < k.
// No permutation passes through LDS between the three transforms.
// D = -1 is the erasure-free case k = n (Sec. II-B): the weights are n^-1
// and the inverse FNT_n alone is the decoder.
template <int LN, int D, int TT, int NT, int VV, class TW>
__device__ __forceinline__ void dec_item(const DecodeArgs& a, uint32_t item, uint32_t* lds, const TW& tws) {
  using Gm = Geo<LN, TT, NT, VV>;
  constexpr int V = Gm::V, G = Gm::G, T = Gm::T;
  const uint32_t tile = item % a.tiles;
  const uint64_t blk = item / a.tiles;
  const uint32_t lane0 = tile * T;
  DecLoad<LN, V> lg{a.recv + blk * a.stride_recv + lane0, a.wfull, a.ridx, a.ld_recv, lane0, a.lanes,
                    a.row0, a.full != 0, a.vec != 0, a.wrb};
  LdsLoad<V, G> ll{lds};
  LdsStore<V, G, false> sl{lds};
  SourceStore<V> sg{a.dst + blk * a.stride_dst + lane0, a.ld_dst, a.k, lane0, a.lanes, a.vec != 0};
  if constexpr (D < 0) {
    dit<LN, Gm::BM, V, G, true>(tws, lg, ll, sl, sg);
  } else {
    constexpr int L2 = LN - D;
    constexpr int BM = Gm::BM;
    constexpr int NP1 = plan_np(LN, BM), NP2 = plan_np(L2, BM);
    LdsStore<V, G, true> slf{lds};
    if constexpr (NP1 >= 2 && NP2 >= 2) {
      // the transforms meet at seams (seam_pass): with M = n, the inverse
      // FNT_n's last pass, the series mask and the DIF's first pass; for any
      // M, the DIF's last pass, the product and the inverse DIT's first pass
      AhatProduct<V> ap{a.ahat_br};
      if constexpr (D == 0) {
        SeriesMask<V> sk{a.k};
        dit_passes<LN, BM, V, G, true, 0, NP1 - 1>(tws, lg, ll, sl);
        seam_pass<LN, BM, V, G, true, true, false>(tws, ll, sk, slf);
        __syncthreads();
        dif_passes<L2, BM, V, G, false, 1, NP2 - 1>(tws, ll, slf);
      } else {
        SeriesStore<V, G> ss{lds, a.k};
        dit<LN, BM, V, G, true>(tws, lg, ll, sl, ss);
        dif_passes<L2, BM, V, G, false, 0, NP2 - 1>(tws, ll, slf);
      }
      seam_pass<L2, BM, V, G, false, false, true>(tws, ll, ap, sl);
      __syncthreads();
      NoHook none;
      dit_from<L2, BM, V, G, true, 1>(tws, ll, sl, sg, none);
    } else {
      SeriesStore<V, G> ss{lds, a.k};
      ProductStore<V, G> sp{lds, a.ahat_br};
      dit<LN, BM, V, G, true>(tws, lg, ll, sl, ss);
      dif<L2, BM, V, G, false>(tws, ll, ll, slf, sp);
      dit<L2, BM, V, G, true>(tws, ll, ll, sl, sg);
    }
  }
}

template <int LN, int D, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_dec(DecodeArgs a) {
  using Gm = Geo<LN, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, a.tw, a.twi);
  dec_item<LN, D, TT, NT, VV>(a, xcd_remap(blockIdx.x, gridDim.x), lds, tws);
}

// Batched decoder: as k_enc_tab, for decode jobs of one code length n and
// one product length M = n / 2^D, each with its own locator.
template <int LN, int D, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_dec_tab(JobTable<DecodeArgs> t, const uint32_t* tw, const uint32_t* twi) {
  using Gm = Geo<LN, TT, NT, VV>;
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, tw, twi);
  for (uint32_t w = xcd_remap(blockIdx.x, gridDim.x); w < t.total; w += gridDim.x) {
    const uint32_t j = find_job(t.start, t.njobs, w);
    const DecodeArgs a = load_global(t.jobs + j);
    dec_item<LN, D, TT, NT, VV>(a, w - gptr(t.start)[j], lds, tws);
    __syncthreads();
  }
}

template <int LN, int TT, int NT, int VV>
__device__ __forceinline__ DecLoad<LN, Geo<LN, TT, NT, VV>::V> dec_loader(const DecodeArgs& a, uint32_t item) {
  constexpr int T = Geo<LN, TT, NT, VV>::T;
  const uint32_t lane0 = (item % a.tiles) * T;
  const uint64_t blk = item / a.tiles;
  return {a.recv + blk * a.stride_recv + lane0, a.wfull, a.ridx, a.ld_recv, lane0, a.lanes, a.row0,
          a.full != 0, a.vec != 0, a.wrb};
}

// Persistent decoder: a grid of resident size walks the work items (numbered
// as in k_dec).  The pass-0 reads of a workgroup's next item (received rows
// and their weights) are issued right before the last pass of the current
// one, so their latency overlaps that pass and its stores; the next item's
// pass 0 then starts from registers.
template <int LN, int D, int TT, int NT, int VV>
__global__ void __launch_bounds__(NT) k_dec_pipe(JobTable<DecodeArgs> t, DecodeArgs one, const uint32_t* tw,
                                                 const uint32_t* twi) {
  using Gm = Geo<LN, TT, NT, VV>;
  constexpr int V = Gm::V, G = Gm::G, T = Gm::T, BM = Gm::BM;
  constexpr int B0 = plan_b(LN, BM, 0);
  constexpr int C0 = pass0_per_thread<LN, BM, G, NT>();
  static_assert(C0 >= 1 && plan_np(LN, BM) >= 2, "pipelined kernel needs whole pass-0 items and two passes");
  using TW = typename Gm::TwType;
  extern __shared__ uint32_t lds[];
  const TW tws = make_tw((const TW*)nullptr, lds + Gm::TILE_BYTES / 4, tw, twi);
  int32_t pre[C0][1 << B0][V];
  uint32_t aux[C0][1 << B0], aux2[C0][1 << B0];   // weights and rows of the current job's positions
  uint32_t w = xcd_remap(blockIdx.x, gridDim.x);
  if (w >= t.total) return;
  uint32_t cjob;
  {
    uint32_t local;
    const DecodeArgs a = job_at(t, one, w, local, cjob);
    auto ld = dec_loader<LN, TT, NT, VV>(a, local);
    consts0<LN, BM, V, G, NT, C0>(ld, aux, aux2);
    prefetch0<LN, BM, V, G, NT, C0>(ld, pre, aux, aux2);
  }
  LdsLoad<V, G> ll{lds};
  LdsStore<V, G, false> sl{lds};
  for (; w < t.total; w += gridDim.x) {
    uint32_t local, job;
    const DecodeArgs a = job_at(t, one, w, local, job);
    auto lg = dec_loader<LN, TT, NT, VV>(a, local);
    const uint32_t lane0 = (local % a.tiles) * T;
    const uint64_t blk = local / a.tiles;
    SourceStore<V> sg{a.dst + blk * a.stride_dst + lane0, a.ld_dst, a.k, lane0, a.lanes, a.vec != 0};
    const uint32_t wn = w + gridDim.x;
    auto hook = [&]() {
      if (wn < t.total) {
        uint32_t ln, jn;
        const DecodeArgs an = job_at(t, one, wn, ln, jn);
        auto ld = dec_loader<LN, TT, NT, VV>(an, ln);
        if (jn != cjob) {
          consts0<LN, BM, V, G, NT, C0>(ld, aux, aux2);
          cjob = jn;
        }
        prefetch0<LN, BM, V, G, NT, C0>(ld, pre, aux, aux2);
      }
    };
    dit_pass0_regs<LN, BM, V, G, NT, C0, true>(tws, lg, pre, aux, aux2, sl);
    __syncthreads();
    if constexpr (D < 0) {
      dit_from<LN, BM, V, G, true, 1>(tws, ll, sl, sg, hook);
    } else {
      LdsStore<V, G, true> slf{lds};
      SeriesStore<V, G> ss{lds, a.k};
      ProductStore<V, G> sp{lds, a.ahat_br};
      NoHook none;
      dit_from<LN, BM, V, G, true, 1>(tws, ll, sl, ss, none);
      __syncthreads();
      dif<LN - D, BM, V, G, false>(tws, ll, ll, slf, sp);
      dit_hooked<LN - D, BM, V, G, true>(tws, ll, ll, sl, sg, hook);
    }
    __syncthreads();   // the next item overwrites the LDS tile
  }
}

}  // namespace ct
}  // namespace fntrs
