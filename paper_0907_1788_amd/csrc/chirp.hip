// libfntrs: evaluation of polynomials on a geometric sequence by one middle
// product (the chirp of Sec. II-B, steps 3 and 5; the middle product of
// Sec. III).
//
// With t_i = i(i-1)/2, t_(i+j) = t_i + t_j + i j, so for any nonzero q
//   c(a q^i) = q^(-t_i) sum_j u_j q^(t_(i+j)),  u_j = c_j a^j q^(-t_j):
// coefficient L-1+i of (u reversed) * v with v_m = q^(t_m), m < L+M-1.  The
// product is cyclic of length P = 2^ceil(log2(L+M-1)), which keeps the
// coefficients L-1 .. L+M-2 exact.  Its three transforms are the encoder's
// (the forward transform of a zero-padded vector); the inverse transform is
// the forward one at negated indices, divided by P.
#include "chirp_kernels.hpp"
#include "field.hpp"
#include "host.hpp"

namespace fntrs {

// the fused kernels, one translation unit per product length 2^L (chirp_inst.hip)
#define FNTRS_CHIRP_DECL(L)                                                          \
  hipError_t chirp_launch_##L(const ChirpArgs& a, uint32_t blocks, hipStream_t s); \
  uint32_t chirp_tile_##L();
FNTRS_CHIRP_DECL(1) FNTRS_CHIRP_DECL(2) FNTRS_CHIRP_DECL(3) FNTRS_CHIRP_DECL(4) FNTRS_CHIRP_DECL(5)
FNTRS_CHIRP_DECL(6) FNTRS_CHIRP_DECL(7) FNTRS_CHIRP_DECL(8) FNTRS_CHIRP_DECL(9) FNTRS_CHIRP_DECL(10)
FNTRS_CHIRP_DECL(11) FNTRS_CHIRP_DECL(12) FNTRS_CHIRP_DECL(13)
#undef FNTRS_CHIRP_DECL
constexpr int kChirpFusedMaxLog = 13;

namespace {

// x^e mod p (e taken mod 65536: x^65536 = 1 for nonzero x).
__device__ __forceinline__ uint32_t fpow(uint32_t x, uint32_t e) {
  e &= 0xFFFFu;
  uint32_t r = 1u;
  while (e) {
    if (e & 1u) r = fmul(r, x);
    x = fmul(x, x);
    e >>= 1;
  }
  return r;
}

__device__ __forceinline__ uint32_t tri_mod(uint32_t i) {   // t_i mod 65536
  const uint64_t t = (uint64_t)i * (i - 1u) / 2u;
  return (uint32_t)(t & 0xFFFFu);
}

// The three sequences of the identity, one word per index:
//   v[m]  = q^(t_m),             m < L + M - 1
//   su[j] = a^j q^(-t_j),        j < L
//   so[i] = q^(-t_i) P^(-1),     i < M
__global__ void k_chirp_tables(uint32_t a, uint32_t q, uint32_t qinv, uint32_t pinv, uint32_t L, uint32_t M,
                               uint32_t* __restrict__ v, uint32_t* __restrict__ su, uint32_t* __restrict__ so) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < L + M - 1) v[m] = fpow(q, tri_mod(m));
  if (m < L) su[m] = fmul(fpow(a, m), fpow(qinv, tri_mod(m)));
  if (m < M) so[m] = fmul(fpow(qinv, tri_mod(m)), pinv);
}

// Row-scaled copies over [batch][rows][lanes]: threads across lanes, rows
// (of every block) across grid.y, grid-stride.  Row `r` of block b is read
// from row src_row(r) and multiplied by scale[r]:
//   kReverse: dst row L-1-r <- src row r     (u, the reversed scaled coefficients)
//   kInPlace: row r *= scale[r]              (the pointwise product with v^)
//   kGather:  dst row r <- src row (P-(L-1+r)) mod P   (the middle coefficients)
enum { kReverse = 0, kInPlace = 1, kGather = 2 };

struct RowScaleArgs {
  const uint32_t* src; uint64_t ld_s, st_s;
  uint32_t* dst; uint64_t ld_d, st_d;
  const uint32_t* scale;
  uint32_t rows, lanes, batch, L, P;
};

template <int kMode>
__global__ void k_chirp_rows(RowScaleArgs a) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.lanes) return;
  const uint32_t total = a.rows * a.batch;
  for (uint32_t rb = blockIdx.y; rb < total; rb += gridDim.y) {
    const uint32_t b = rb / a.rows, r = rb - b * a.rows;
    const uint32_t w = a.scale[r];
    uint32_t sr = r, dr = r;
    if (kMode == kReverse) dr = a.L - 1 - r;
    if (kMode == kGather) sr = (a.P - (a.L - 1 + r) % a.P) % a.P;
    const uint32_t x = a.src[b * a.st_s + (uint64_t)sr * a.ld_s + l];
    a.dst[b * a.st_d + (uint64_t)dr * a.ld_d + l] = fmul(x, w);
  }
}

// vbr[p] = vhat[bitrev(p)], p < 2^logp.
__global__ void k_chirp_perm(const uint32_t* __restrict__ vhat, uint32_t* __restrict__ vbr, int logp) {
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < (1u << logp)) vbr[p] = vhat[bitrev(p, logp)];
}

struct ChirpFused {
  hipError_t (*launch)(const ChirpArgs&, uint32_t, hipStream_t);
  uint32_t (*tile)();
};
const ChirpFused& chirp_fused(int logp) {
  static const ChirpFused t[kChirpFusedMaxLog + 1] = {
      {nullptr, nullptr},               {chirp_launch_1, chirp_tile_1},   {chirp_launch_2, chirp_tile_2},
      {chirp_launch_3, chirp_tile_3},   {chirp_launch_4, chirp_tile_4},   {chirp_launch_5, chirp_tile_5},
      {chirp_launch_6, chirp_tile_6},   {chirp_launch_7, chirp_tile_7},   {chirp_launch_8, chirp_tile_8},
      {chirp_launch_9, chirp_tile_9},   {chirp_launch_10, chirp_tile_10}, {chirp_launch_11, chirp_tile_11},
      {chirp_launch_12, chirp_tile_12}, {chirp_launch_13, chirp_tile_13}};
  return t[logp];
}

uint32_t P_of(uint64_t len) { return std::max<uint32_t>(2, pad_pow2((uint32_t)len)); }

uint32_t host_pow(uint32_t x, uint32_t e) {
  uint64_t r = 1, b = x % 65537u;
  while (e) {
    if (e & 1u) r = r * b % 65537u;
    b = b * b % 65537u;
    e >>= 1;
  }
  return (uint32_t)r;
}

}  // namespace
}  // namespace fntrs

using namespace fntrs;

extern "C" int fntrs_chirp_eval(fntrs_ctx* c, uint32_t L, uint32_t M, uint32_t a, uint32_t q, const uint32_t* coeffs,
                                size_t ld_in, size_t stride_in, uint32_t* out, size_t ld_out, size_t stride_out,
                                uint32_t lanes, uint32_t batch, void* stream) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (L < 1 || M < 1 || lanes < 1 || batch < 1) return fail(c, FNTRS_E_INVAL, "L, M, lanes and batch must be >= 1");
  if (!coeffs || !out) return fail(c, FNTRS_E_INVAL, "null coeffs or out");
  if (a == 0 || q == 0 || a > 65536 || q > 65536)
    return fail(c, FNTRS_E_INVAL, "a=%u and q=%u must be nonzero residues", a, q);
  if (ld_in < lanes || ld_out < lanes) return fail(c, FNTRS_E_INVAL, "ld_in/ld_out smaller than lanes");
  if (batch > 1 && (stride_in < (size_t)(L - 1) * ld_in + lanes || stride_out < (size_t)(M - 1) * ld_out + lanes))
    return fail(c, FNTRS_E_INVAL, "block strides overlap consecutive blocks");
  const uint64_t len = (uint64_t)L + M - 1;
  if (len > 65536)
    return fail(c, FNTRS_E_UNSUPPORTED, "L + M - 1 = %llu exceeds the longest transform, 65536",
                (unsigned long long)len);
  if ((uint64_t)P_of(len) * batch > 0xFFFFFFFFull) return fail(c, FNTRS_E_INVAL, "batch %u too large", batch);
  const size_t ib = span_elems(batch, stride_in, L, ld_in, lanes) * 4, ob = span_elems(batch, stride_out, M, ld_out,
                                                                                     lanes) * 4;
  if (ranges_overlap(coeffs, ib, out, ob)) return fail(c, FNTRS_E_INVAL, "coeffs and out overlap");
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  const uint32_t P = P_of(len);
  const uint32_t qinv = host_pow(q, 65535), pinv = host_pow(P, 65535);
  if (ilog2(P) <= kChirpFusedMaxLog) {
    // fused: tables v, v^, v^ bit-reversed, su, so (P words each), then one
    // kernel over (lane tile, block)
    const int logp = ilog2(P);
    const size_t vw = (P + 63) / 64 * 64;
    const uint32_t T = chirp_fused(logp).tile();
    const uint64_t blocks = (uint64_t)((lanes + T - 1) / T) * batch;
    if (blocks > 0x7fffffffull) return fail(c, FNTRS_E_INVAL, "grid too large");
    Scratch sc;
    if (int rc = scratch_acquire(c, 5 * vw * 4, s, sc)) return rc;
    uint32_t* v = reinterpret_cast<uint32_t*>(sc.p);
    uint32_t* vhat = v + vw;
    uint32_t* vbr = vhat + vw;
    uint32_t* su = vbr + vw;
    uint32_t* so = su + vw;
    int rc = FNTRS_OK;
    hipLaunchKernelGGL(k_chirp_tables, dim3((uint32_t)((len + 255) / 256)), dim3(256), 0, s, a, q, qinv, pinv, L, M,
                       v, su, so);
    if (hipGetLastError() != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "chirp table kernel");
    if (!rc) rc = encode_run(c, P, (uint32_t)len, 1, v, 1, P, vhat, 1, P, 1, 0, s);
    if (!rc) {
      hipLaunchKernelGGL(k_chirp_perm, dim3((P + 255) / 256), dim3(256), 0, s, (const uint32_t*)vhat, vbr, logp);
      if (hipGetLastError() != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "chirp permutation kernel");
    }
    if (!rc) {
      ChirpArgs ca{};
      ca.c = coeffs; ca.ld_c = ld_in; ca.st_c = stride_in;
      ca.out = out; ca.ld_o = ld_out; ca.st_o = stride_out;
      ca.su = su; ca.so = so; ca.vhat_br = vbr; ca.tw = c->tw; ca.twi = c->twi;
      ca.L = L; ca.M = M; ca.lanes = lanes; ca.tiles = (lanes + T - 1) / T;
      ca.vec = aligned16(coeffs, ld_in, stride_in) && aligned16(out, ld_out, stride_out);
      if (chirp_fused(logp).launch(ca, (uint32_t)blocks, s) != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "chirp kernel");
    }
    scratch_release(c, sc, s);
    return rc;
  }
  // P > 2^13: three transforms through HBM.  Scratch: v and its transform
  // (P words each), the two scale tables, u and its transform (batch x P x
  // lanes each)
  const size_t vw = (P + 63) / 64 * 64, uw = (size_t)batch * P * lanes;
  Scratch sc;
  if (int rc = scratch_acquire(c, (4 * vw + 2 * uw) * 4, s, sc)) return rc;
  uint32_t* v = reinterpret_cast<uint32_t*>(sc.p);
  uint32_t* vhat = v + vw;
  uint32_t* su = vhat + vw;
  uint32_t* so = su + vw;
  uint32_t* u = so + vw;
  uint32_t* uhat = u + uw;
  const size_t ld_u = lanes, st_u = (size_t)P * lanes;
  int rc = FNTRS_OK;
  hipLaunchKernelGGL(k_chirp_tables, dim3((uint32_t)((len + 255) / 256)), dim3(256), 0, s, a, q, qinv, pinv, L, M,
                     v, su, so);
  if (hipGetLastError() != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "chirp table kernel");
  if (!rc) rc = encode_run(c, P, (uint32_t)len, 1, v, 1, P, vhat, 1, P, 1, 0, s);
  auto rows = [&](int mode, const uint32_t* src, uint64_t ld_s, uint64_t st_s, uint32_t* dst, uint64_t ld_d,
                  uint64_t st_d, const uint32_t* scale, uint32_t nrows, const char* what) {
    RowScaleArgs r{src, ld_s, st_s, dst, ld_d, st_d, scale, nrows, lanes, batch, L, P};
    const dim3 grid((lanes + 255) / 256, (uint32_t)std::min<uint64_t>((uint64_t)nrows * batch, 65535));
    if (mode == kReverse) hipLaunchKernelGGL(k_chirp_rows<kReverse>, grid, dim3(256), 0, s, r);
    else if (mode == kInPlace) hipLaunchKernelGGL(k_chirp_rows<kInPlace>, grid, dim3(256), 0, s, r);
    else hipLaunchKernelGGL(k_chirp_rows<kGather>, grid, dim3(256), 0, s, r);
    return hipGetLastError() == hipSuccess ? FNTRS_OK : fail(c, FNTRS_E_DEVICE, "chirp %s kernel", what);
  };
  if (!rc) rc = rows(kReverse, coeffs, ld_in, stride_in, u, ld_u, st_u, su, L, "scaling");
  if (!rc) rc = encode_run(c, P, L, lanes, u, ld_u, st_u, uhat, ld_u, st_u, batch, 0, s);
  if (!rc) rc = rows(kInPlace, uhat, ld_u, st_u, uhat, ld_u, st_u, vhat, P, "product");
  // the inverse transform: the forward one (into u) read at negated indices
  if (!rc) rc = encode_run(c, P, P, lanes, uhat, ld_u, st_u, u, ld_u, st_u, batch, 0, s);
  if (!rc) rc = rows(kGather, u, ld_u, st_u, out, ld_out, stride_out, so, M, "output");
  scratch_release(c, sc, s);
  return rc;
}
