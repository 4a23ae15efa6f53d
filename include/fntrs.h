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

/* Pseudo-device for fntrs_create: a context that touches no GPU.  Every call
 * on it runs the full host-side argument validation and, if the arguments
 * pass, returns FNTRS_E_DEVICE without doing any work. */
#define FNTRS_HOST_ONLY (-1)

/* Create a context on HIP device `device` (or FNTRS_HOST_ONLY).  It owns the
 * twiddle table (powers of the primitive root 3, Sec. II-A), the locator
 * cache and scratch memory; `workspace_cap_bytes` caps that memory
 * (0 = 4 GiB).  On success *out receives the context.  Errors: FNTRS_E_INVAL
 * (null out, bad device), FNTRS_E_DEVICE, FNTRS_E_NOMEM. */
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
 * n: power of two in [1, 65536]; 1 <= k <= n (any k, zero padding covers a k
 * that is not a power of two, Sec. II-B); lanes >= 1; batch >= 1 blocks.
 * src and dst must not overlap.  Errors: FNTRS_E_INVAL, FNTRS_E_DEVICE,
 * FNTRS_E_RANGE (validate flag). */
int fntrs_encode(fntrs_ctx* ctx, uint32_t n, uint32_t k, uint32_t lanes,
                 const uint32_t* src, size_t ld_src, size_t stride_src,
                 uint32_t* dst, size_t ld_dst, size_t stride_dst,
                 uint32_t batch, uint32_t flags, void* stream);

/* Locator for one erasure pattern (Sec. II-B, steps 1-3, which depend only
 * on the received positions and are reused for every lane and block).
 * positions: host array of npos received positions in [0, n), strictly
 * ascending; the first k are used (Sec. II-B: "the first k evaluation
 * points received").  Builds on the device, enqueued on `stream`:
 *   A(x) = prod_{i<k} (x - r_n^(z_i)) by a product tree of FNT products,
 *   A'(x), its values at the received points by FNT_n, their inverses,
 *   and the FNT of size 2k of the low coefficients of A.
 * A pattern already in the context's cache is returned without rebuilding.
 * *out receives a reference that must be given back with
 * fntrs_locator_release.  k must be a power of two (k = n is allowed: no
 * erasure).  Errors: FNTRS_E_INVAL, FNTRS_E_TOOFEW (npos < k),
 * FNTRS_E_POSITIONS, FNTRS_E_UNSUPPORTED (k not a power of two),
 * FNTRS_E_NOMEM, FNTRS_E_DEVICE. */
int fntrs_locator(fntrs_ctx* ctx, uint32_t n, uint32_t k,
                  const uint32_t* positions, uint32_t npos,
                  void* stream, fntrs_locator_t** out);

/* Give back a locator reference.  The state stays cached for reuse until the
 * context needs the memory; work already enqueued that uses it is not
 * affected.  Errors: FNTRS_E_INVAL. */
int fntrs_locator_release(fntrs_ctx* ctx, fntrs_locator_t* loc);

/* Copy a locator's state to host memory (synchronous; for inspection and
 * tests).  Any pointer may be NULL.  A: k+1 coefficients of A(x), lowest
 * first; w: k values 1/A'(x_i); ahat: 2k values FNT_2k(a_0..a_(k-1),0..0) in
 * natural order.  For k = n only A is meaningful (x^n - 1).  Returns
 * FNTRS_OK, FNTRS_E_INVAL or FNTRS_E_DEVICE. */
int fntrs_locator_export(fntrs_ctx* ctx, const fntrs_locator_t* loc,
                         uint32_t* A, uint32_t* w, uint32_t* ahat);

/* Decoder (Sec. II-B, steps 4-6): recovers the k source rows of every block
 * from the k received symbols of the locator's pattern.  flags selects the
 * recv layout (FNTRS_RECV_COMPACT: k rows in position order; FNTRS_RECV_FULL:
 * n rows, row z read for each received position z) and may add
 * FNTRS_FLAG_VALIDATE.  dst receives k rows per block.  recv and dst must not
 * overlap.  Errors: FNTRS_E_INVAL, FNTRS_E_DEVICE, FNTRS_E_RANGE. */
int fntrs_decode(fntrs_ctx* ctx, const fntrs_locator_t* loc, uint32_t lanes, uint32_t flags,
                 const uint32_t* recv, size_t ld_recv, size_t stride_recv,
                 uint32_t* dst, size_t ld_dst, size_t stride_dst,
                 uint32_t batch, void* stream);

/* Library version string. */
const char* fntrs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FNTRS_H */
