/*
 * fntrs -- FNT-based Reed-Solomon erasure coding over GF(65537) on AMD MI355X.
 *
 * C ABI of libfntrs.so.  Only plain pointers, integers and sizes cross this
 * boundary; the library is written in HIP for gfx950.
 *
 * The code (Soro & Lacan, "FNT-based Reed-Solomon Erasure Codes"):
 *   p = 65537, n = 2^i <= 65536, r_n = 3^(65536/n) (Sec. II-B, root choice).
 *   Encoding maps k source symbols s_0..s_(k-1) to n encoded symbols
 *   e_i = s(r_n^i), i = 0..n-1, i.e. the FNT of (s, 0, ..., 0) (Sec. II-B).
 *   Any k of the n encoded symbols recover s (MDS, Sec. I and II-A); the
 *   decoder interpolates through the received points with the six-step
 *   algorithm of Sec. II-B.
 *
 * Data layout shared by every entry point.  A "block" is one codeword of
 * symbols; every symbol is a row of `lanes` 16-bit lanes, each lane stored
 * as a uint32 residue in [0, 65536], lane index fastest:
 *     element (block b, row i, lane l) is at ptr[b*stride + i*ld + l]
 * Each lane is an independent codeword (the paper applies the code to every
 * 16-bit lane of a packet or file chunk, Sec. II-B).  `ld` (elements between
 * rows, >= lanes) and `stride` (elements between blocks) are counted in
 * uint32 elements.  Data pointers are device pointers owned by the caller.
 *
 * Asynchrony.  encode / locator / decode validate their arguments on the host,
 * synchronously, then enqueue GPU work on `stream` (a hipStream_t passed as
 * void*, NULL = the null stream) and return.  Inputs must stay valid, and
 * outputs must not be read, until the stream reaches the call.
 *
 * Input residues must lie in [0, 65536]; larger values give unspecified (but
 * deterministic) results unless FNTRS_FLAG_VALIDATE is set, in which case the
 * call reads the inputs back and returns FNTRS_E_RANGE.
 *
 * Thread safety: one context may be used from several host threads; calls on
 * one context are serialised by an internal lock.
 */
#ifndef FNTRS_H
#define FNTRS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fntrs_ctx fntrs_ctx;
typedef struct fntrs_locator_s fntrs_locator_t;

enum {
  FNTRS_OK = 0,
  FNTRS_E_INVAL = -1,       /* bad size, null pointer, ld < lanes, ...        */
  FNTRS_E_TOOFEW = -2,      /* fewer than k received positions (Sec. II-B)    */
  FNTRS_E_POSITIONS = -3,   /* duplicate, unsorted or out-of-range position   */
  FNTRS_E_RANGE = -4,       /* an input residue > 65536 (validate mode only)  */
  FNTRS_E_NOMEM = -5,       /* device memory or the context's cap exhausted   */
  FNTRS_E_DEVICE = -6,      /* a HIP runtime error; see fntrs_last_error      */
  FNTRS_E_UNSUPPORTED = -7  /* a size this build does not implement           */
};

/* decode flags */
#define FNTRS_RECV_COMPACT 0u   /* recv holds k rows: row i is the symbol received at positions[i] */
#define FNTRS_RECV_FULL 1u      /* recv holds n rows indexed by position; only the k received rows are read */
#define FNTRS_FLAG_VALIDATE 2u  /* check input residues <= 65536 first (synchronous) */
/* encode and decode flag: the systematic code of Sec. II-C (single calls
 * only; a batched job with this flag is rejected with FNTRS_E_UNSUPPORTED) */
#define FNTRS_SYSTEMATIC 4u
/* encode and decode flag: the direct (quadratic) methods of Sec. III instead
 * of the transforms, for k <= 1024 and n <= 16384 (else FNTRS_E_UNSUPPORTED;
 * decoding also needs k < n).  The result is the same, bit for bit; only the
 * cost differs: a product with a fixed matrix, O(n k) per lane to encode and
 * O(k^2) to decode, which on small codes does in one kernel what the
 * transforms do in several passes.
 *   encode:                 dst = G src, G[i][j] = r_N^(i j)
 *   encode | SYSTEMATIC:    dst rows 0..k-1 = src, rows k..n-1 = C src, C the
 *                           Lagrange basis of positions 0..k-1 evaluated at
 *                           the other positions (Table I, direct encoding;
 *                           C is built once per (n, k) and kept)
 *   decode:                 dst = W v, W the inverse of the generator's rows
 *                           at the received positions (built once per
 *                           locator and kept with it)
 *   decode | SYSTEMATIC:    the received source positions are copied and only
 *                           the missing ones computed (Table II, direct
 *                           decoding)
 * Single calls only: a batched job with this flag is rejected. */
#define FNTRS_DIRECT 8u
/* encode and decode flag: always the transforms, even for a class the
 * autotuner gave to the direct methods. */
#define FNTRS_TRANSFORM 16u

/* Pseudo-device for fntrs_create: a context that touches no GPU.  Every call
 * on it runs the full host-side argument validation and, if the arguments
 * pass, returns FNTRS_E_DEVICE without doing any work. */
#define FNTRS_HOST_ONLY (-1)

/* Create a context on HIP device `device` (or FNTRS_HOST_ONLY).  It owns the
 * twiddle table (powers of the primitive root 3, Sec. II-A), the locator
 * cache and scratch memory; `workspace_cap_bytes` (0 = 4 GiB) caps the
 * locator cache, and separately the device blocks the context keeps for
 * reuse as scratch (four-step passes, batch tables, locator builds).  A call
 * whose scratch fits in no kept block under the cap allocates it
 * stream-ordered instead.  Kept blocks are reused in stream order: a call on
 * another stream first waits (on the device) for the block's last use.  On
 * success *out receives the context.  Errors: FNTRS_E_INVAL (null out, bad
 * device), FNTRS_E_DEVICE, FNTRS_E_NOMEM. */
int fntrs_create(int device, size_t workspace_cap_bytes, fntrs_ctx** out);

/* Destroy a context: waits for the device, frees everything it owns,
 * including locators not yet released.  NULL is ignored. */
void fntrs_destroy(fntrs_ctx* ctx);

/* Text of the last error recorded on this context ("" if none).  The string
 * is owned by the context and valid until its next call. */
const char* fntrs_last_error(const fntrs_ctx* ctx);

/* Encoder (Sec. II-B): for every block b, row i < n and lane l < lanes,
 *     dst[b][i][l] = sum_{j<k} src[b][j][l] * r_n^(i*j)  (mod 65537),
 * the FNT of size n of the zero-padded source.  src holds k rows, dst n rows.
 * n in [1, 65536]; a length that is not a power of two is read as puncturing
 * (Sec. II-B): the code of length N, the next power of two, with rows
 * n..N-1 neither computed into dst nor sent (r_N takes the place of r_n);
 * 1 <= k <= n (any k, zero padding covers a k that is not a power of two,
 * Sec. II-B); lanes >= 1; batch >= 1 blocks.
 * src and dst must not overlap.
 * flags: 0, FNTRS_FLAG_VALIDATE, FNTRS_SYSTEMATIC and/or FNTRS_DIRECT.  With
 * FNTRS_SYSTEMATIC the systematic code of Sec. II-C: the source is
 * interpolated on positions 0..k-1 into k intermediate symbols (the decoder,
 * with the locator of that pattern, which the context builds once and
 * caches), and dst is the transform above of the intermediate symbols, so
 * that dst rows 0..k-1 equal src; the call holds batch*k*lanes words of
 * the context's scratch, ordered on `stream`.
 * Errors: FNTRS_E_INVAL, FNTRS_E_DEVICE, FNTRS_E_RANGE (validate flag),
 * FNTRS_E_NOMEM, FNTRS_E_UNSUPPORTED. */
int fntrs_encode(fntrs_ctx* ctx, uint32_t n, uint32_t k, uint32_t lanes,
                 const uint32_t* src, size_t ld_src, size_t stride_src,
                 uint32_t* dst, size_t ld_dst, size_t stride_dst,
                 uint32_t batch, uint32_t flags, void* stream);

/* The encoder of fntrs_encode for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and the same result, bit for bit, but the
 * call allocates nothing.  Where the encoder needs a scratch buffer (k above
 * 8192, i.e. transforms of 2^14 points or more, run as four-step passes) it
 * uses a fixed array in device memory that the library holds on every GPU it
 * runs on until the process ends: at most 2^25 words (128 MiB), i.e.
 * batch * N * (lanes rounded up to 32) <= 33554432 with N the next power of
 * two >= n (k = 16384, n = 32768: up to 1024 lanes x blocks; n = 65536: up
 * to 512).  Every call on one GPU shares that array, so calls that overlap
 * on one GPU race: enqueue them on one stream, or order their streams.
 * flags must be 0 (FNTRS_FLAG_VALIDATE and FNTRS_SYSTEMATIC allocate).
 * Errors: those of fntrs_encode; FNTRS_E_NOMEM when the scratch would exceed
 * the fixed array (nothing is enqueued). */
int fntrs_encode_noalloc(fntrs_ctx* ctx, uint32_t n, uint32_t k, uint32_t lanes,
                         const uint32_t* src, size_t ld_src, size_t stride_src,
                         uint32_t* dst, size_t ld_dst, size_t stride_dst,
                         uint32_t batch, uint32_t flags, void* stream);

/* Locator for one erasure pattern (Sec. II-B, steps 1-3, which depend only
 * on the received positions and are reused for every lane and block).
 * positions: host array of npos received positions in [0, n), strictly
 * ascending; only the first k of them are used (Sec. II-B, decoding from
 * the earliest k received points).  n in [1, 65536], as for fntrs_encode (a punctured
 * length uses the points of the next power of two).  Builds on the device,
 * enqueued on `stream`:
 *   A(x) = prod_{i<k} (x - r_n^(z_i)) by a product tree of FNT products,
 *   A'(x), its values at the received points by FNT_n, their inverses,
 *   and the FNT of size 2k of the low coefficients of A.
 * A pattern of 2^12 positions or more built alone (this call, or a batch of
 * one) takes the same quantities from discrete logarithms instead: one
 * cyclic convolution of the received-position indicator with
 * log(r_n^d - 1), exact over GF(65537) bit plane by bit plane, gives
 * log A(x_j) and log A'(x_z) at every point, hence the weights and the
 * transform of A mod x^k; the coefficients of A are then taken on first
 * use (fntrs_locator_export, the direct decoder).  The first such pattern
 * of a given n builds a table of 16 n words, kept with the context (the
 * call synchronises `stream` once for it).
 * A pattern already in the context's cache is returned without rebuilding.
 * *out receives a reference that must be given back with
 * fntrs_locator_release.  Any 1 <= k <= n (k = n is allowed: no erasure); a
 * k that is not a power of two runs the product tree on the next power of
 * two with the extra roots at 0 and divides their factor out.  Errors:
 * FNTRS_E_INVAL, FNTRS_E_TOOFEW (npos < k), FNTRS_E_POSITIONS,
 * FNTRS_E_UNSUPPORTED (k < N with 2K > N, N and K the powers of two at or
 * above n and k: the low product would be longer than the transform; this
 * includes 32768 < k < n), FNTRS_E_NOMEM, FNTRS_E_DEVICE. */
int fntrs_locator(fntrs_ctx* ctx, uint32_t n, uint32_t k,
                  const uint32_t* positions, uint32_t npos,
                  void* stream, fntrs_locator_t** out);

/* Locators of `count` erasure patterns at once: pattern q has code length
 * n[q], k[q] source symbols and npos[q] received positions at positions[q]
 * (host memory, the rules of fntrs_locator).  Patterns not in the cache are
 * built together, one launch per stage for all of them (O(log k) launches
 * in total instead of per pattern; a single launch when every pattern has
 * erasures and n <= 1024), and share one device allocation that is
 * returned when the last of them leaves the cache.  out[q] receives a
 * reference as from fntrs_locator (release each).  All or nothing: on error
 * no reference is returned and fntrs_last_error names the pattern.  Errors:
 * those of fntrs_locator. */
int fntrs_locator_batch(fntrs_ctx* ctx, uint32_t count, const uint32_t* n, const uint32_t* k,
                        const uint32_t* const* positions, const uint32_t* npos,
                        void* stream, fntrs_locator_t** out);

/* Give back a locator reference.  The state stays cached for reuse until the
 * context needs the memory; work already enqueued that uses it is not
 * affected.  Errors: FNTRS_E_INVAL. */
int fntrs_locator_release(fntrs_ctx* ctx, fntrs_locator_t* loc);

/* Copy a locator's state to host memory (synchronous; for inspection and
 * tests).  Any pointer may be NULL.  A: k+1 coefficients of A(x), lowest
 * first; w: k values 1/A'(x_i); ahat: 2k values FNT_2k(a_0..a_(k-1),0..0) in
 * natural order, written only when k is a power of two (the transform of
 * length 2k exists only then).  For k = n only A is meaningful (x^n - 1).  Returns
 * FNTRS_OK, FNTRS_E_INVAL or FNTRS_E_DEVICE. */
int fntrs_locator_export(fntrs_ctx* ctx, const fntrs_locator_t* loc,
                         uint32_t* A, uint32_t* w, uint32_t* ahat);

/* Decoder (Sec. II-B, steps 4-6): recovers the k source rows of every block
 * from the k received symbols of the locator's pattern.  flags selects the
 * recv layout (FNTRS_RECV_COMPACT: k rows in position order; FNTRS_RECV_FULL:
 * n rows, row z read for each received position z) and may add
 * FNTRS_FLAG_VALIDATE.  dst receives k rows per block.  recv and dst must not
 * overlap.  With FNTRS_SYSTEMATIC (Sec. II-C) the received symbols are those
 * of a systematic codeword (fntrs_encode with FNTRS_SYSTEMATIC): the decoder
 * recovers the k intermediate symbols and transforms them at positions
 * 0..k-1, so dst receives the source; the call holds batch*k*lanes words
 * of the context's scratch, ordered on `stream`.
 * Errors: FNTRS_E_INVAL, FNTRS_E_DEVICE, FNTRS_E_RANGE, FNTRS_E_NOMEM. */
int fntrs_decode(fntrs_ctx* ctx, const fntrs_locator_t* loc, uint32_t lanes, uint32_t flags,
                 const uint32_t* recv, size_t ld_recv, size_t stride_recv,
                 uint32_t* dst, size_t ld_dst, size_t stride_dst,
                 uint32_t batch, void* stream);

/* Evaluation of polynomials on a geometric sequence by one middle product
 * (the chirp of Sec. II-B, step 3, which also serves step 5; the middle
 * product of Sec. III): for every block b, point i < M and lane l,
 *     out[b][i][l] = sum_{j<L} coeffs[b][j][l] * (a q^i)^j   (mod 65537),
 * i.e. each lane holds the L coefficients of one polynomial, lowest degree
 * first.  With t_i = i(i-1)/2 the values are q^(-t_i) times the middle
 * coefficients L-1 .. L+M-2 of the product of (c_j a^j q^(-t_j)) reversed by
 * (q^(t_m)), computed as a cyclic product of length P = 2^ceil(log2(L+M-1)):
 * three transforms of the encoder and three pointwise kernels.  Step 3
 * evaluates A' on positions in arithmetic progression (q = r_n^d,
 * a = r_n^s); step 5's S_j = -N'(r_n^(-j-1)) is q = a = r_n^-1.  a and q:
 * nonzero residues; L + M - 1 <= 65536.  Device pointers; asynchronous on
 * `stream`; uses 4 P + 2 batch P lanes words of context scratch.
 * Errors: FNTRS_E_INVAL, FNTRS_E_UNSUPPORTED (L + M - 1 > 65536),
 * FNTRS_E_NOMEM, FNTRS_E_DEVICE. */
int fntrs_chirp_eval(fntrs_ctx* ctx, uint32_t L, uint32_t M, uint32_t a, uint32_t q, const uint32_t* coeffs,
                     size_t ld_in, size_t stride_in, uint32_t* out, size_t ld_out, size_t stride_out,
                     uint32_t lanes, uint32_t batch, void* stream);

/* 16-bit transport of encoding symbols (Sec. II-B: every residue but 65536
 * is a 16-bit value; the positions holding 65536 travel in the symbol's
 * header).  A symbol is one row of `lanes` residues; in/out hold `rows` rows
 * per block, `batch` blocks, row-major with the given row pitch (ld) and
 * block pitch (stride), in elements.  All pointers are device memory; the
 * calls are asynchronous on `stream`.
 *
 * fntrs_pack16: out[b][r][l] = in[b][r][l] mod 65536 (65536 is sent as 0);
 * esc_count[b*rows + r] = the number of lanes of row r of block b holding
 * 65536, and esc_pos[(b*rows + r)*esc_cap + i], i < min(count, esc_cap),
 * those lanes in ascending order (esc_cap = lanes always suffices; a row
 * with more than esc_cap of them still reports its full count, and only
 * the first esc_cap positions are written).  Inputs must be residues in
 * [0, 65536].
 * fntrs_unpack16: the inverse: out = in widened, and the first
 * min(esc_count, esc_cap) listed lanes of each row set to 65536.
 * lanes <= 65536.  Errors: FNTRS_E_INVAL, FNTRS_E_DEVICE. */
int fntrs_pack16(fntrs_ctx* ctx, const uint32_t* in, size_t ld_in, size_t stride_in, uint32_t rows,
                 uint32_t lanes, uint32_t batch, uint16_t* out, size_t ld_out, size_t stride_out,
                 uint32_t* esc_count, uint32_t* esc_pos, uint32_t esc_cap, void* stream);
int fntrs_unpack16(fntrs_ctx* ctx, const uint16_t* in, size_t ld_in, size_t stride_in, uint32_t rows,
                   uint32_t lanes, uint32_t batch, const uint32_t* esc_count, const uint32_t* esc_pos,
                   uint32_t esc_cap, uint32_t* out, size_t ld_out, size_t stride_out, void* stream);

/* ------------------------------------------------------------------------
 * Batched path: uneven batches of encode and decode jobs.
 *
 * A job carries the arguments of one fntrs_encode or fntrs_decode call.  Its
 * result is bit-identical to that call's: the batch changes how the work is
 * launched, not what is computed.  Jobs of one size class (encode: transform
 * size K = 2^ceil(log2 k); decode: code length n and product length) share
 * one persistent launch whose workgroups walk a device-side table of the
 * class's jobs; the classes run concurrently on internal streams of default
 * priority and are joined back into the caller's stream.
 * ------------------------------------------------------------------------ */

#define FNTRS_OP_ENCODE 0u
#define FNTRS_OP_DECODE 1u

typedef struct fntrs_job {
  uint32_t op;                 /* FNTRS_OP_ENCODE or FNTRS_OP_DECODE */
  uint32_t n, k;               /* encode: code length and source symbols (the
                                  rules of fntrs_encode); decode: 0, or equal
                                  to the locator's n and k */
  uint32_t lanes, batch;       /* lanes per row, codeword blocks */
  uint32_t flags;              /* encode: 0; decode: FNTRS_RECV_COMPACT or
                                  FNTRS_RECV_FULL (FNTRS_FLAG_VALIDATE is
                                  rejected: it would synchronise the batch;
                                  FNTRS_SYSTEMATIC is not batched) */
  const fntrs_locator_t* loc;  /* decode: locator of the received positions;
                                  encode: NULL */
  const uint32_t* in;          /* encode: src [batch][k][ld_in];
                                  decode: recv [batch][k or n][ld_in] */
  size_t ld_in, stride_in;
  uint32_t* out;               /* encode: dst [batch][n][ld_out];
                                  decode: dst [batch][k][ld_out] */
  size_t ld_out, stride_out;
} fntrs_job;

/* Enqueue `njobs` jobs on `stream` (asynchronous, like the single calls).
 * The job array is read before the call returns; data buffers and locators
 * must stay valid until the stream reaches the batch.  Every job is checked
 * as its single call would be; in addition no job's output may overlap any
 * other job's input or output.  A working buffer for the job tables and the
 * scratch of four-step jobs (2^14 points or more; the ones given to one
 * stream run one after another over that stream's slice) is allocated
 * stream-ordered and freed after the batch.  Errors: FNTRS_E_INVAL (with the
 * job index in fntrs_last_error), FNTRS_E_NOMEM, FNTRS_E_DEVICE. */
int fntrs_submit(fntrs_ctx* ctx, const fntrs_job* jobs, uint32_t njobs, void* stream);

/* A batch captured once into a HIP graph and replayed many times on the same
 * buffers (whose contents may change between replays).  The graph owns its
 * job tables and scratch (counted against the context's cap) and holds a
 * reference to every locator it reads until it is destroyed. */
typedef struct fntrs_graph_s fntrs_graph_t;

/* Checks and plans the batch as fntrs_submit does, then captures it.  The
 * kernel configuration of each size class is frozen at capture time.
 * Errors: as fntrs_submit; FNTRS_E_INVAL also for an empty batch. */
int fntrs_graph_create(fntrs_ctx* ctx, const fntrs_job* jobs, uint32_t njobs, fntrs_graph_t** out);

/* Replays the batch on `stream` (after the builds of its locators). */
int fntrs_graph_launch(fntrs_ctx* ctx, fntrs_graph_t* graph, void* stream);

/* Frees the graph (waits for replays in flight) and its locator references. */
int fntrs_graph_destroy(fntrs_ctx* ctx, fntrs_graph_t* graph);

/* Kernel configuration of one transform size. */
typedef struct fntrs_tuning {
  uint32_t tile_lanes;        /* lanes per workgroup tile */
  uint32_t threads;           /* threads per workgroup */
  uint32_t lanes_per_thread;  /* lanes one thread carries through a pass */
  uint32_t radix_log2;        /* largest radix of the LDS passes, as log2 */
  float ms;                   /* autotune: mean time of the chosen configuration per launch */
  uint32_t op;                /* FNTRS_OP_ENCODE or FNTRS_OP_DECODE */
  uint32_t log2_size;         /* transform size class: encode log2 K, decode log2 N */
  uint32_t method;            /* FNTRS_METHOD_TRANSFORM, _DIRECT or _FOURSTEP */
  float default_ms;           /* autotune: the default configuration's time */
} fntrs_tuning;

#define FNTRS_METHOD_TRANSFORM 0u   /* one-pass-per-tile transform kernels */
#define FNTRS_METHOD_DIRECT 1u      /* the quadratic methods of Sec. III (FNTRS_DIRECT) */
#define FNTRS_METHOD_FOURSTEP 2u    /* four-step transforms (2^14 points or more) */

/* Autotuner for single calls: times every compiled configuration of the size
 * class of (op, n, k) on `lanes` x `batch` scratch codewords, `reps` calls
 * each (synchronous), and makes the fastest the context's configuration for
 * that class, used by later single calls, batches and graphs.  For codes the
 * direct methods cover (k <= 1024, n <= 16384, and k < n to decode) it also
 * times FNTRS_DIRECT and, if that is faster, makes later non-systematic
 * single calls of the class without FNTRS_DIRECT or FNTRS_TRANSFORM use it.
 * Any 1 <= k <= n <= 65536; four-step classes (2^14 points or more) have one
 * configuration, which is timed and reported.  Errors: FNTRS_E_INVAL,
 * FNTRS_E_UNSUPPORTED, FNTRS_E_NOMEM, FNTRS_E_DEVICE. */
int fntrs_autotune(fntrs_ctx* ctx, uint32_t op, uint32_t n, uint32_t k, uint32_t lanes, uint32_t batch,
                   uint32_t reps, void* stream, fntrs_tuning* chosen);

/* Autotuner for a batch: for every size class of the table kernels in the
 * batch (encode by K, decode by N), runs the class's own jobs, `reps` times
 * per compiled configuration, and keeps the fastest as the context's
 * configuration; four-step classes are timed with their one configuration.
 * The batch's buffers are written (outputs) but inputs are only read.
 * Synchronous.  out[0 .. *nout) receives one entry per class (at most cap).
 * Errors: those of fntrs_submit. */
int fntrs_autotune_batch(fntrs_ctx* ctx, const fntrs_job* jobs, uint32_t njobs, uint32_t reps, void* stream,
                         fntrs_tuning* out, uint32_t cap, uint32_t* nout);

/* Current configuration of transform size 2^log2_size (1..15) for op. */
int fntrs_get_config(fntrs_ctx* ctx, uint32_t op, uint32_t log2_size, fntrs_tuning* cfg);

/* Library version string. */
const char* fntrs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FNTRS_H */
