// Kernel argument structs of the coding and locator kernels: plain data
// (pointers and sizes) that the host fills in and passes by value or through
// device-side tables.
#pragma once
#include <cstddef>
#include <cstdint>

namespace fntrs {

struct EncodeArgs {
  const uint32_t* src;
  uint64_t ld_src, stride_src;
  uint32_t* dst;
  uint64_t ld_dst, stride_dst;
  const uint32_t* tw;        // tw[e] = 3^e
  const uint32_t* twi;       // twi[e] = 3^-e
  uint32_t n, k, lanes;
  int logn, logK;            // transform size K = 2^logK >= k, K <= n
  uint32_t tiles, cosets;    // lane tiles per block, n / K
  uint32_t vec;              // src/dst rows are 16-byte aligned (vector access allowed)
  uint32_t rows_out;         // only rows i < rows_out of dst are written (0: all n)
};

struct DecodeArgs {
  const uint32_t* recv;
  uint64_t ld_recv, stride_recv;
  uint32_t* dst;
  uint64_t ld_dst, stride_dst;
  const uint32_t* tw;
  const uint32_t* twi;
  const uint32_t* wfull;    // per position z < n: decoder weight (0 if z is erased)
  const uint32_t* ridx;     // per position z < n: row of z in a compact recv
  const uint32_t* ahat_br;  // FNT_M of A's low part, bit-reversed order, times M^-1
  uint32_t n, k, lanes;
  int logn, logk;
  uint32_t full;            // recv holds n rows indexed by position
  uint32_t tiles, vec;
  uint32_t row0;            // a received row of recv: erased positions read it and discard the value
  // optional: (weight, row) of position bitrev(p) at wrb[2p], p < n, the
  // order the first pass reads them in (row 0 where the weight is 0); null:
  // the first pass reads wfull and ridx
  const uint32_t* wrb;
};

// Work table of the batched path: the jobs of one class (one transform size,
// one kernel configuration) share a persistent launch; job j owns the work
// items [start[j], start[j+1]), numbered as the single-job grid numbers its
// workgroups.
template <class Args>
struct JobTable {
  const Args* jobs;
  const uint32_t* start;    // njobs + 1 ascending entries, start[0] = 0
  uint32_t njobs, total;    // total = start[njobs]
};

struct FourStepArgs {
  const uint32_t* in;       // first-pass input (recv / src) or scratch
  uint64_t ld_in, stride_in;
  uint32_t* out;            // scratch or final output
  uint64_t ld_out, stride_out;
  const uint32_t* tw;       // 3^e
  const uint32_t* twi;      // 3^-e
  const uint32_t* wfull;    // decoder weights per position
  const uint32_t* ridx;     // compact recv row per position
  const uint32_t* ahat;     // FNT_M(A mod x^k) / M, natural order
  uint32_t n, k, M, lanes;
  int logn, logm;
  uint32_t full, tiles, subs, vec;   // subs: sub-transforms per block
  uint32_t rows_out;                 // encoder: only rows < rows_out of out are written (0: all n)
  uint64_t tstride_in, tstride_out;  // elements between lane tiles (set by the four-step launchers)
  uint64_t foff_in, foff_out;        // scratch in / out: byte offset of its bit-16 flags (four-step launchers)
  uint32_t order;                    // work item order (fs::work_of): 0 tile first, 1 sub-transform
                                     // first, 2 sub-transform pairs, then tiles
  // scratch in / out: byte offset of the escape bitmap (one bit per row of a
  // lane tile, set where a lane holds 65536; see fs::scratch_put), log2 of
  // the rows per tile, and (out) log2 of the writer's row split S: its rows
  // are i*S + m, and row i*S + m has bit m*(R/S) + i of its tile's R bits
  uint64_t boff_in, boff_out;
  uint32_t rlog_in, rlog_out, slog_out;
  const uint32_t* wr;                // decoder K1: weights and rows by sub-transform (FsPrepArgs::wr)
  const uint32_t* twsplit;           // this kernel's split twiddles by [sub-transform][index]
  const uint32_t* ahat_t;            // decoder K3: the locator's transform by [sub-transform][index]
};

// Layout of the context's twiddle allocation, in words from its start:
// tw[e] = 3^e (e < 65536), then twi[e] = 3^-e, then the tables of every
// transform stage, omega_(2^lg)^j = 3^(j 2^(16-lg)) for j <= 2^(lg-1) and
// lg = 1..16 one after another (a workgroup fills its LDS stage tables from
// consecutive words instead of words 2^(16-lg) apart), then the four-step
// split twiddles (split_tw_offset).
constexpr size_t kStageTwBase = 2 * size_t(65536);
constexpr uint32_t stage_tw_offset(int lg) { return ((1u << (lg - 1)) - 1) + (lg - 1); }
constexpr size_t kStageTwWords = stage_tw_offset(17);

// The first launch of a four-step call: the escape bitmaps it clears before
// the call's kernels run (up to three ranges of whole 16-byte vectors) and,
// for the decoder, the tables it lays out for K1 and K3.
struct FsPrepArgs {
  uint32_t* p[3];
  uint64_t words[3];   // multiples of 4
  // decoder: the weight and row of input i2 of K1's sub-transform i1 (the
  // position z = i1 + (n/256) i2), as word pairs at wr[2 (256 i1 + i2)]
  // (null: none); the row is 0 where the weight is 0
  uint32_t* wr;
  const uint32_t* wfull;
  const uint32_t* ridx;
  uint32_t n, full;
  // decoder: ahat (natural order, M words) laid out for K3 as
  // ahat_t[256 m2' + j] = ahat[m2' + (M/256) j] (null: none)
  uint32_t* ahat_t;
  const uint32_t* ahat;
  uint32_t M;
};

// One erasure pattern of a locator batch: where its positions come from,
// where its state goes, its scratch, its sizes.
struct LocDesc {
  const uint32_t* zin;      // the k received positions (batch upload)
  uint32_t* pos;            // state: positions, k words
  uint32_t* wfull;          // state: decoder weight per position, n words
  uint32_t* ridx;           // state: compact row per position, n words
  uint32_t* ahat_br;        // state: FNT_M(A mod x^k) / M, bit-reversed, M words
  uint32_t* ahat_s;         // state: the same in natural order, M words
  uint32_t* A;              // state: A(x), k+1 coefficients
  uint32_t* w;              // state: 1/A'(x_i), k words
  uint32_t* ahat;           // state: FNT_M(A mod x^k), M words
  uint32_t* t0;             // scratch: product-tree levels, k words each
  uint32_t* t1;
  uint32_t* spec;           // scratch: parked transforms, then A', k words
  uint32_t* vals;           // scratch: A' at every n-th root, n words
  uint32_t* poly;           // t0 or t1: where the tree leaves A mod x^k
  uint32_t n, k, G;         // k: points of the product tree (a power of two); G points per leaf
  uint32_t kr;              // received positions (k rounded up to the tree is padded with roots at 0)
  int logn, logk, logm;
};

// One short-code pattern passed whole as a kernel argument (k_locb_small1):
// its descriptor and its received positions (n <= 1024 gives k <= 512).
constexpr uint32_t kLocSmallMaxK = 512;
struct LocSmallOne {
  LocDesc d;
  uint32_t z[kLocSmallMaxK];
};

// Last pass of the logarithmic locator of one large pattern (k_conv_finish).
struct ConvFinishArgs {
  const uint32_t* Q;      // forward FNT_n of the 16 products, [n][16]
  const uint32_t* ind;    // indicator of R
  const uint32_t* ridx;   // rank of each received position
  const uint32_t* tw;     // 3^e, e < 65536
  uint32_t* w;            // state: 1/A'(x_z) by rank
  uint32_t* wfull;        // state: decoder weight per position
  uint32_t* ahat;         // state: FNT_M(A mod x^k), natural
  uint32_t* ahat_br;      // state: the same / M, bit-reversed
  uint32_t* ahat_s;       // state: the same / M, natural
  uint32_t* vals;         // A(x_j) for every j (0 on R)
  uint32_t S, kr;
  int logn, logm;
};

// Direct (quadratic) methods: Y[b][yrow(r)][l] = sum_j M(r, j) X[b][xrow(j)][l]
// mod p, r < R, j < K, l < lanes.  M(r, j) is M[r*ldm + j], or (M null)
// r_N^(pw(r) j) from the table 3^e, with pw(r) = pw[r] (or r when pw is
// null); null row maps are the identity.
struct GemmArgs {
  const uint32_t* M;
  uint64_t ldm;
  const uint32_t* pw;
  const uint32_t* tw;
  int logN;
  const uint32_t* X;
  uint64_t ld_x, stride_x;
  const uint32_t* xrow;
  uint32_t* Y;
  uint64_t ld_y, stride_y;
  const uint32_t* yrow;
  uint32_t R, K, lanes;
};

}  // namespace fntrs
