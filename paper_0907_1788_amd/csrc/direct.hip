// libfntrs: the direct (quadratic) encoders and decoders of Sec. III.
//
// Every direct method is a product of a fixed matrix with the k rows of each
// block, Y = M X mod p, per lane:
//   non-systematic encode:  M = G, G[i][j] = r_N^(i j)          (n x k)
//   non-systematic decode:  M = W = V_R^-1                       (k x k)
//   systematic encode:      parity rows k..n-1 = C s, C = G_par W_0
//                           (Table I, direct encoding)
//   systematic decode:      missing source rows s_E = D v, D = G_E W_R
//                           (Table II, direct decoding)
// W_R (the inverse of the received rows of the generator) has column i equal
// to w_i A(x)/(x - x_i), whose coefficients come from A by synthetic
// division; A and w are the locator's (steps 1-3 of Sec. II-B).  W_0 is the
// same for the positions 0..k-1.
//
// These are dense contractions, so they run on the matrix cores, in double
// precision: residues are at most 2^16, so every product is an integer below
// 2^32 and a sum of up to 2^20 of them is exact in a double's 53-bit
// mantissa.  One reduction mod p per output.
#include "field.hpp"
#include "host.hpp"

namespace fntrs {

namespace {

// One wave computes a 16 x 16 tile of Y (16 rows r, 16 lanes l) with the
// double-precision matrix instruction D += A B, A 16 x 4 (M), B 4 x 16 (X):
// lane t supplies A[t % 16][t / 16] and B[t / 16][t % 16] and holds
// D[4 i + t / 16][t % 16], i < 4 (the lane layout measured on gfx950).  K advances 4 per instruction; the
// operands of kKU instructions are loaded before they run.
constexpr int kKU = 8;
static_assert(kDirectMaxK <= 4 * 256, "the inverse-Vandermonde builder holds 4 terms per thread");

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t mod_p(double acc) {
  const uint64_t v = (uint64_t)acc;   // exact: acc is a non-negative integer below 2^53
  return (uint32_t)(v % 65537ull);
}

// Operand values of K-step u for this lane (0 past the edges).
struct GemmLane {
  const GemmArgs& a;
  const uint32_t* X;
  const uint32_t* mrow;
  uint32_t p, Nmask, l, tk;
  bool rok, lok;
  __device__ __forceinline__ void load(uint32_t k0, uint32_t (&m)[kKU], uint32_t (&x)[kKU]) const {
#pragma unroll
    for (int u = 0; u < kKU; ++u) {
      const uint32_t k = k0 + 4 * u + tk;
      m[u] = 0;
      x[u] = 0;
      if (k < a.K) {
        if (rok) m[u] = mrow ? mrow[k] : a.tw[((p * k) & Nmask) << (16 - a.logN)];
        if (lok) x[u] = X[(uint64_t)(a.xrow ? a.xrow[k] : k) * a.ld_x + l];
      }
    }
  }
};

__global__ void __launch_bounds__(64) k_gemm_modp(GemmArgs a) {
  const uint32_t t = threadIdx.x, tc = t % 16, tk = t / 16;
  const uint32_t l0 = blockIdx.x * 16, r0 = blockIdx.y * 16;
  const uint64_t b = blockIdx.z;
  const uint32_t r = r0 + tc, l = l0 + tc;   // the A row and the B column this lane supplies
  const bool rok = r < a.R, lok = l < a.lanes;
  const GemmLane g{a, a.X + b * a.stride_x, (rok && a.M) ? a.M + (uint64_t)r * a.ldm : nullptr,
                   (rok && !a.M) ? (a.pw ? a.pw[r] : r) : 0u, (1u << a.logN) - 1u, l, tk, rok, lok};
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  // the loads of the next kKU steps are in flight while this group's products run
  uint32_t m[kKU], x[kKU], mn[kKU], xn[kKU];
  g.load(0, m, x);
  for (uint32_t k0 = 0; k0 < a.K; k0 += 4 * kKU) {
    if (k0 + 4 * kKU < a.K) g.load(k0 + 4 * kKU, mn, xn);
#pragma unroll
    for (int u = 0; u < kKU; ++u)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64((double)m[u], (double)x[u], acc, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < kKU; ++u) {
      m[u] = mn[u];
      x[u] = xn[u];
    }
  }
  uint32_t* Y = a.Y + b * a.stride_y;
  const uint32_t lo = l0 + tc;
  if (lo >= a.lanes) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t ro = r0 + 4 * i + tk;
    if (ro < a.R) Y[(uint64_t)(a.yrow ? a.yrow[ro] : ro) * a.ld_y + lo] = mod_p(acc[i]);
  }
}

// W[j][i] = w_i * (coefficient j of A(x)/(x - x_i)), one workgroup per
// column i.  Synthetic division gives coefficient j of A(x)/(x - x_i) as
// q_j = sum_{m > j} a_m x_i^(m-j-1) = x_i^(-j-1) S_j with the suffix sums
// S_j = sum_{m > j} a_m x_i^m (a_k = 1): every term is independent (x_i^m is
// one table lookup, x_i being a power of the root), and S is a suffix scan.
constexpr int kIVT = 256;
__global__ void __launch_bounds__(kIVT) k_inv_vandermonde(const uint32_t* __restrict__ A,
                                                         const uint32_t* __restrict__ w,
                                                         const uint32_t* __restrict__ pos,
                                                         const uint32_t* __restrict__ tw,
                                                         const uint32_t* __restrict__ twi, int logN, uint32_t k,
                                                         uint32_t* __restrict__ W) {
  __shared__ uint32_t part[kIVT];
  const uint32_t i = blockIdx.x, t = threadIdx.x;
  const uint32_t sh = 16 - logN, Nmask = (1u << logN) - 1u;
  const uint32_t z = pos[i];
  // thread t owns terms m = 1 + t*c .. t*c + c (c per thread), suffix-summed locally
  const uint32_t c = (k + kIVT - 1) / kIVT;
  uint32_t loc[4];   // c <= 4 (k <= 1024)
  uint32_t run = 0;
  for (int u = (int)c - 1; u >= 0; --u) {
    const uint32_t m = 1 + t * c + (uint32_t)u;
    const uint32_t term = m <= k ? fmul(A[m], tw[((z * m) & Nmask) << sh]) : 0u;
    run = fadd(run, term);
    loc[u] = run;
  }
  part[t] = run;
  __syncthreads();
  // suffix scan of the thread totals: part[t] = sum over threads >= t
  for (uint32_t d = 1; d < kIVT; d <<= 1) {
    const uint32_t v = t + d < kIVT ? part[t + d] : 0u;
    __syncthreads();
    part[t] = fadd(part[t], v);
    __syncthreads();
  }
  const uint32_t after = t + 1 < kIVT ? part[t + 1] : 0u;
  const uint32_t wi = w[i];
  for (uint32_t u = 0; u < c; ++u) {
    const uint32_t m = 1 + t * c + u;   // S_(m-1) = sum of terms >= m
    if (m > k) break;
    const uint32_t j = m - 1;
    const uint32_t S = fadd(loc[u], after);
    const uint32_t xinv = twi[((z * (j + 1)) & Nmask) << sh];   // x_i^(-j-1)
    W[(uint64_t)j * k + i] = fmul(wi, fmul(S, xinv));
  }
}

// dst[b][drow[r]][l] = src[b][srow[r]][l] for r < rows (source rows that were
// received, copied by the systematic direct decoder); null maps: row r.
__global__ void k_copy_rowmap(const uint32_t* __restrict__ src, uint64_t ld_s, uint64_t st_s,
                              const uint32_t* __restrict__ srow, uint32_t* __restrict__ dst, uint64_t ld_d,
                              uint64_t st_d, const uint32_t* __restrict__ drow, uint32_t rows, uint32_t lanes) {
  const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t r = blockIdx.y;
  const uint64_t b = blockIdx.z;
  if (l >= lanes || r >= rows) return;
  dst[b * st_d + (uint64_t)(drow ? drow[r] : r) * ld_d + l] = src[b * st_s + (uint64_t)(srow ? srow[r] : r) * ld_s + l];
}

hipError_t gemm(const GemmArgs& a, uint32_t batch, hipStream_t s) {
  if (!a.R || !a.lanes || !batch) return hipSuccess;
  if (a.R > 16u * 65535u) return hipErrorInvalidValue;
  const dim3 grid((a.lanes + 15) / 16, (a.R + 15) / 16, batch);
  hipLaunchKernelGGL(k_gemm_modp, grid, dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// A device buffer holding a matrix of the direct methods (W of a locator, or
// the context's parity matrix of a systematic code), built on some stream;
// users wait on `ready`.
struct DirectMat {
  uint32_t* p = nullptr;
  size_t bytes = 0;
  hipEvent_t ready = nullptr;
};

size_t direct_mat_bytes(const DirectMat* m) { return m ? m->bytes : 0; }

void direct_mat_free(DirectMat* m) {
  if (!m) return;
  if (m->ready) (void)hipEventDestroy(m->ready);
  if (m->p) (void)hipFree(m->p);   // waits for work still using it
  delete m;
}

namespace {

int direct_mat_alloc(fntrs_ctx* c, size_t words, DirectMat*& out) {
  out = nullptr;
  if (!make_room(c, words * 4))
    return fail(c, FNTRS_E_NOMEM, "direct-method matrix of %zu bytes exceeds the context cap", words * 4);
  auto* m = new DirectMat();
  if (hipMalloc((void**)&m->p, words * 4) != hipSuccess) {
    delete m;
    return fail(c, FNTRS_E_NOMEM, "hipMalloc(%zu) for a direct-method matrix failed", words * 4);
  }
  m->bytes = words * 4;
  if (hipEventCreateWithFlags(&m->ready, hipEventDisableTiming) != hipSuccess) {
    direct_mat_free(m);
    return fail(c, FNTRS_E_DEVICE, "event creation failed");
  }
  c->used += m->bytes;
  out = m;
  return FNTRS_OK;
}

// W = V_R^-1 of a locator (k x k), built once on the first direct decode.
int locator_inverse(fntrs_ctx* c, fntrs_locator_t* L, hipStream_t s, const DirectMat*& out) {
  if (!L->direct_w) {
    if (int rc = locator_coeffs(c, L, s)) return rc;   // reads A
    DirectMat* m = nullptr;
    if (int rc = direct_mat_alloc(c, (size_t)L->k * L->k, m)) return rc;
    HIP_TRY(c, hipStreamWaitEvent(s, L->ready, 0));
    hipLaunchKernelGGL(k_inv_vandermonde, dim3(L->k), dim3(kIVT), 0, s, L->A, L->w, L->pos, c->tw, c->twi, L->logn,
                       L->k, m->p);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) {
      direct_mat_free(m);
      c->used -= (size_t)L->k * L->k * 4;
      return fail(c, FNTRS_E_DEVICE, "inverse Vandermonde kernel: %s", hipGetErrorString(e));
    }
    HIP_TRY(c, hipEventRecord(m->ready, s));
    L->direct_w = m;
  }
  HIP_TRY(c, hipStreamWaitEvent(s, L->direct_w->ready, 0));
  out = L->direct_w;
  return FNTRS_OK;
}

GemmArgs data_args(const uint32_t* X, size_t ld_x, size_t st_x, uint32_t* Y, size_t ld_y, size_t st_y,
                   uint32_t lanes) {
  GemmArgs a{};
  a.X = X; a.ld_x = ld_x; a.stride_x = st_x;
  a.Y = Y; a.ld_y = ld_y; a.stride_y = st_y;
  a.lanes = lanes;
  return a;
}

}  // namespace

bool direct_fits(uint32_t N, uint32_t k) { return k >= 1 && k <= kDirectMaxK && N <= kDirectMaxN; }

// Non-systematic direct encoder: dst rows i < rows = sum_j r_N^(i j) src_j.
int direct_encode(fntrs_ctx* c, uint32_t N, uint32_t rows, uint32_t k, uint32_t lanes, const uint32_t* src,
                  size_t ld_src, size_t stride_src, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
                  hipStream_t s) {
  GemmArgs a = data_args(src, ld_src, stride_src, dst, ld_dst, stride_dst, lanes);
  a.tw = c->tw; a.logN = ilog2(N);
  a.R = rows; a.K = k;
  HIP_TRY(c, gemm(a, batch, s));
  return FNTRS_OK;
}

// Non-systematic direct decoder: s = W v over the locator's k received rows.
int direct_decode(fntrs_ctx* c, fntrs_locator_t* L, uint32_t lanes, bool full, const uint32_t* recv, size_t ld_recv,
                  size_t stride_recv, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch, hipStream_t s) {
  const DirectMat* W = nullptr;
  if (int rc = locator_inverse(c, L, s, W)) return rc;
  GemmArgs a = data_args(recv, ld_recv, stride_recv, dst, ld_dst, stride_dst, lanes);
  a.M = W->p; a.ldm = L->k;
  a.xrow = full ? L->pos : nullptr;
  a.R = L->k; a.K = L->k;
  HIP_TRY(c, gemm(a, batch, s));
  return FNTRS_OK;
}

// Systematic direct encoder (Sec. III, Table I): rows 0..k-1 of dst are the
// source, rows k..rows-1 are C s with C = G_par W_0, cached per (N, k).
int direct_systematic_encode(fntrs_ctx* c, uint32_t N, uint32_t rows, uint32_t k, uint32_t lanes,
                             const uint32_t* src, size_t ld_src, size_t stride_src, uint32_t* dst, size_t ld_dst,
                             size_t stride_dst, uint32_t batch, hipStream_t s) {
  const uint32_t npar = rows - k;
  if (npar) {
    const auto key = std::make_pair(N, k);
    auto it = c->parity.find(key);
    if (it == c->parity.end()) {
      // W_0 from the locator of positions 0..k-1 (cached in the context)
      std::vector<uint32_t> first(k);
      for (uint32_t i = 0; i < k; ++i) first[i] = i;
      const uint32_t* fp = first.data();
      fntrs_locator_t* L0 = nullptr;
      if (int rc = locators_acquire(c, 1, &N, &k, &fp, &k, s, &L0)) return rc;
      const DirectMat* W0 = nullptr;
      int rc = locator_inverse(c, L0, s, W0);
      DirectMat* C = nullptr;
      if (!rc) rc = direct_mat_alloc(c, (size_t)(N - k) * k, C);
      if (!rc) {
        // C[t][j] = sum_m x_(k+t)^m W_0[m][j]: W_0 enters as a block of k rows of k lanes
        std::vector<uint32_t> pw(N - k);
        for (uint32_t t = 0; t < N - k; ++t) pw[t] = k + t;
        uint32_t* dpw = nullptr;
        if (hipMallocAsync((void**)&dpw, pw.size() * 4, s) != hipSuccess) {
          rc = fail(c, FNTRS_E_NOMEM, "row table");
        } else {
          rc = upload_async(c, dpw, pw.data(), pw.size() * 4, s);
          GemmArgs a = data_args(W0->p, k, (size_t)k * k, C->p, k, (size_t)(N - k) * k, k);
          a.tw = c->tw; a.logN = ilog2(N); a.pw = dpw;
          a.R = N - k; a.K = k;
          if (!rc && gemm(a, 1, s) != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "parity matrix product");
          (void)hipFreeAsync(dpw, s);
          if (!rc && hipEventRecord(C->ready, s) != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "event record");
        }
        if (rc) {
          c->used -= C->bytes;
          direct_mat_free(C);
          C = nullptr;
        }
      }
      L0->refs--;
      if (rc) return rc;
      it = c->parity.emplace(key, C).first;
    }
    HIP_TRY(c, hipStreamWaitEvent(s, it->second->ready, 0));
    GemmArgs a = data_args(src, ld_src, stride_src, dst + (size_t)k * ld_dst, ld_dst, stride_dst, lanes);
    a.M = it->second->p; a.ldm = k;
    a.R = npar; a.K = k;
    HIP_TRY(c, gemm(a, batch, s));
  }
  // the source rows themselves
  hipLaunchKernelGGL(k_copy_rowmap, dim3((lanes + 255) / 256, k, batch), dim3(256), 0, s, src, (uint64_t)ld_src,
                     (uint64_t)stride_src, (const uint32_t*)nullptr, dst, (uint64_t)ld_dst, (uint64_t)stride_dst,
                     (const uint32_t*)nullptr, k, lanes);
  HIP_TRY(c, hipGetLastError());
  return FNTRS_OK;
}

// Systematic direct decoder (Sec. III, Table II): the received source rows
// (positions < k) are copied; the missing ones are D v with D = G_E W_R, E
// the missing source positions, built once per locator.
int direct_systematic_decode(fntrs_ctx* c, fntrs_locator_t* L, uint32_t lanes, bool full, const uint32_t* recv,
                             size_t ld_recv, size_t stride_recv, uint32_t* dst, size_t ld_dst, size_t stride_dst,
                             uint32_t batch, hipStream_t s) {
  const uint32_t k = L->k;
  if (!L->direct_sys) {
    // E: source positions not among the k received; R0: received ones, with their recv row
    std::vector<uint32_t> tab;   // [E (e)] [R0 positions (g)] [R0 recv rows (g)]
    std::vector<uint32_t> got;
    std::vector<uint8_t> seen(k, 0);
    for (uint32_t i = 0; i < k; ++i)
      if (L->positions[i] < k) seen[L->positions[i]] = 1;
    for (uint32_t m = 0; m < k; ++m)
      if (!seen[m]) tab.push_back(m);
    const uint32_t e = (uint32_t)tab.size();
    for (uint32_t i = 0; i < k; ++i)
      if (L->positions[i] < k) tab.push_back(L->positions[i]);
    const uint32_t g = (uint32_t)tab.size() - e;
    for (uint32_t i = 0; i < k; ++i)
      if (L->positions[i] < k) tab.push_back(i);
    DirectMat* m = nullptr;
    if (int rc = direct_mat_alloc(c, (size_t)e * k + tab.size() + 64, m)) return rc;
    uint32_t* D = m->p;
    uint32_t* dtab = m->p + (size_t)e * k;
    int rc = upload_async(c, dtab, tab.data(), tab.size() * 4, s);
    if (!rc && e) {
      const DirectMat* W = nullptr;
      rc = locator_inverse(c, L, s, W);
      if (!rc) {
        GemmArgs a = data_args(W->p, k, (size_t)k * k, D, k, (size_t)e * k, k);
        a.tw = c->tw; a.logN = L->logn; a.pw = dtab;
        a.R = e; a.K = k;
        if (gemm(a, 1, s) != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "decoding matrix product");
      }
    }
    if (!rc && hipEventRecord(m->ready, s) != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "event record");
    if (rc) {
      c->used -= m->bytes;
      direct_mat_free(m);
      return rc;
    }
    L->direct_sys = m;
    L->direct_e = e;
    L->direct_g = g;
  }
  HIP_TRY(c, hipStreamWaitEvent(s, L->direct_sys->ready, 0));
  const uint32_t e = L->direct_e, g = L->direct_g;
  const uint32_t* dtab = L->direct_sys->p + (size_t)e * k;
  if (e) {
    GemmArgs a = data_args(recv, ld_recv, stride_recv, dst, ld_dst, stride_dst, lanes);
    a.M = L->direct_sys->p; a.ldm = k;
    a.xrow = full ? L->pos : nullptr;
    a.yrow = dtab;
    a.R = e; a.K = k;
    HIP_TRY(c, gemm(a, batch, s));
  }
  if (g) {
    const uint32_t* srow = full ? dtab + e : dtab + e + g;   // full: row = position; compact: the recv row
    hipLaunchKernelGGL(k_copy_rowmap, dim3((lanes + 255) / 256, g, batch), dim3(256), 0, s, recv, (uint64_t)ld_recv,
                       (uint64_t)stride_recv, srow, dst, (uint64_t)ld_dst, (uint64_t)stride_dst, dtab + e, g, lanes);
    HIP_TRY(c, hipGetLastError());
  }
  return FNTRS_OK;
}

}  // namespace fntrs
