// libfntrs: host side of the C ABI declared in include/fntrs.h.
//
// Validation happens here, synchronously, before anything is enqueued; the
// coding work itself runs in the compile-time kernels (ct_kernels.hpp, one
// translation unit per transform size) and the locator kernels
// (locator_kernels.hpp).  The batched path (jobs, graphs, autotuning) is in
// submit.hip.
#include "host.hpp"
#include "locator_kernels.hpp"

namespace fntrs {

int fail(fntrs_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

// Launch tables of the per-size translation units, indexed by log2 size.
const CtTables& ct_tables() {
  static const CtEncLaunch enc[16] = {nullptr, ct_enc_launch_1, ct_enc_launch_2, ct_enc_launch_3, ct_enc_launch_4,
                                 ct_enc_launch_5, ct_enc_launch_6, ct_enc_launch_7, ct_enc_launch_8,
                                 ct_enc_launch_9, ct_enc_launch_10, ct_enc_launch_11, ct_enc_launch_12,
                                 ct_enc_launch_13, ct_enc_launch_14, ct_enc_launch_15};
  static const CtDecLaunch dec[16] = {nullptr, ct_dec_launch_1, ct_dec_launch_2, ct_dec_launch_3, ct_dec_launch_4,
                                 ct_dec_launch_5, ct_dec_launch_6, ct_dec_launch_7, ct_dec_launch_8,
                                 ct_dec_launch_9, ct_dec_launch_10, ct_dec_launch_11, ct_dec_launch_12,
                                 ct_dec_launch_13, ct_dec_launch_14, ct_dec_launch_15};
  static const CtEncTabLaunch enc_tab[16] = {
    nullptr,              ct_enc_tab_launch_1,  ct_enc_tab_launch_2,  ct_enc_tab_launch_3,
    ct_enc_tab_launch_4,  ct_enc_tab_launch_5,  ct_enc_tab_launch_6,  ct_enc_tab_launch_7,
    ct_enc_tab_launch_8,  ct_enc_tab_launch_9,  ct_enc_tab_launch_10, ct_enc_tab_launch_11,
    ct_enc_tab_launch_12, ct_enc_tab_launch_13, ct_enc_tab_launch_14, ct_enc_tab_launch_15};
  static const CtDecTabLaunch dec_tab[16] = {
    nullptr,              ct_dec_tab_launch_1,  ct_dec_tab_launch_2,  ct_dec_tab_launch_3,
    ct_dec_tab_launch_4,  ct_dec_tab_launch_5,  ct_dec_tab_launch_6,  ct_dec_tab_launch_7,
    ct_dec_tab_launch_8,  ct_dec_tab_launch_9,  ct_dec_tab_launch_10, ct_dec_tab_launch_11,
    ct_dec_tab_launch_12, ct_dec_tab_launch_13, ct_dec_tab_launch_14, ct_dec_tab_launch_15};
  static const CtTabOccupancy occ[16] = {
    nullptr,             ct_tab_occupancy_1,  ct_tab_occupancy_2,  ct_tab_occupancy_3,
    ct_tab_occupancy_4,  ct_tab_occupancy_5,  ct_tab_occupancy_6,  ct_tab_occupancy_7,
    ct_tab_occupancy_8,  ct_tab_occupancy_9,  ct_tab_occupancy_10, ct_tab_occupancy_11,
    ct_tab_occupancy_12, ct_tab_occupancy_13, ct_tab_occupancy_14, ct_tab_occupancy_15};
  static const CtTables t{enc, dec, enc_tab, dec_tab, occ};
  return t;
}

int check_encode(fntrs_ctx* c, uint32_t n, uint32_t k, uint32_t lanes, const uint32_t* src, size_t ld_src,
                 size_t stride_src, const uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
                 uint32_t flags) {
  if (!is_pow2(n) || n > 65536) return fail(c, FNTRS_E_INVAL, "n=%u must be a power of two in [1, 65536]", n);
  if (k < 1 || k > n) return fail(c, FNTRS_E_INVAL, "k=%u must satisfy 1 <= k <= n=%u", k, n);
  if (lanes < 1 || batch < 1) return fail(c, FNTRS_E_INVAL, "lanes=%u and batch=%u must be >= 1", lanes, batch);
  if (!src || !dst) return fail(c, FNTRS_E_INVAL, "null src or dst");
  if (ld_src < lanes || ld_dst < lanes) return fail(c, FNTRS_E_INVAL, "ld_src/ld_dst smaller than lanes");
  if (batch > 1 && (stride_src < (size_t)(k - 1) * ld_src + lanes || stride_dst < (size_t)(n - 1) * ld_dst + lanes))
    return fail(c, FNTRS_E_INVAL, "block strides overlap consecutive blocks");
  if (flags & ~FNTRS_FLAG_VALIDATE) return fail(c, FNTRS_E_INVAL, "unknown flags 0x%x", flags);
  const size_t sb = span_elems(batch, stride_src, k, ld_src, lanes) * 4;
  const size_t db = span_elems(batch, stride_dst, n, ld_dst, lanes) * 4;
  if (ranges_overlap(src, sb, dst, db)) return fail(c, FNTRS_E_INVAL, "src and dst overlap");
  return FNTRS_OK;
}

int check_decode(fntrs_ctx* c, const fntrs_locator_t* L, uint32_t lanes, uint32_t flags, const uint32_t* recv,
                 size_t ld_recv, size_t stride_recv, const uint32_t* dst, size_t ld_dst, size_t stride_dst,
                 uint32_t batch) {
  if (!L) return fail(c, FNTRS_E_INVAL, "null locator");
  if (L->refs <= 0) return fail(c, FNTRS_E_INVAL, "locator was released");
  if (lanes < 1 || batch < 1) return fail(c, FNTRS_E_INVAL, "lanes=%u and batch=%u must be >= 1", lanes, batch);
  if (!recv || !dst) return fail(c, FNTRS_E_INVAL, "null recv or dst");
  if (flags & ~(FNTRS_RECV_FULL | FNTRS_FLAG_VALIDATE)) return fail(c, FNTRS_E_INVAL, "unknown flags 0x%x", flags);
  const bool full = flags & FNTRS_RECV_FULL;
  const uint32_t n = L->n, k = L->k;
  const uint32_t rrows = full ? n : k;
  if (ld_recv < lanes || ld_dst < lanes) return fail(c, FNTRS_E_INVAL, "ld_recv/ld_dst smaller than lanes");
  if (batch > 1 && (stride_recv < (size_t)(rrows - 1) * ld_recv + lanes || stride_dst < (size_t)(k - 1) * ld_dst + lanes))
    return fail(c, FNTRS_E_INVAL, "block strides overlap consecutive blocks");
  const size_t rb = span_elems(batch, stride_recv, rrows, ld_recv, lanes) * 4;
  const size_t db = span_elems(batch, stride_dst, k, ld_dst, lanes) * 4;
  if (ranges_overlap(recv, rb, dst, db)) return fail(c, FNTRS_E_INVAL, "recv and dst overlap");
  return FNTRS_OK;
}

namespace {

uint64_t hash_positions(uint32_t n, uint32_t k, const uint32_t* z) {
  uint64_t h = 0xcbf29ce484222325ull ^ ((uint64_t)n << 32) ^ k;
  for (uint32_t i = 0; i < k; ++i) {
    h ^= z[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

hipError_t set_lds_attr(const void* fn, size_t bytes) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

int validate_range(fntrs_ctx* c, const uint32_t* p, uint32_t batch, size_t stride, uint32_t rows,
                   size_t ld, uint32_t lanes, hipStream_t s) {
  const size_t cnt = span_elems(batch, stride, rows, ld, lanes);
  std::vector<uint32_t> h(cnt);
  HIP_TRY(c, hipStreamSynchronize(s));
  HIP_TRY(c, hipMemcpy(h.data(), p, cnt * 4, hipMemcpyDeviceToHost));
  for (uint32_t b = 0; b < batch; ++b)
    for (uint32_t r = 0; r < rows; ++r)
      for (uint32_t l = 0; l < lanes; ++l) {
        const uint32_t v = h[b * stride + r * ld + l];
        if (v > 65536u)
          return fail(c, FNTRS_E_RANGE, "input residue %u > 65536 at block %u row %u lane %u", v, b, r, l);
      }
  return FNTRS_OK;
}

static void free_locator(fntrs_ctx* c, fntrs_locator_t* L) {
  if (L->ready) (void)hipEventDestroy(L->ready);
  if (L->mem) {
    (void)hipFree(L->mem);
    c->used -= L->bytes;
  }
  delete L;
}

// Least recently used first.
bool make_room(fntrs_ctx* c, size_t need) {
  while (c->used + need > c->cap) {
    auto victim = c->cache.end();
    for (auto it = c->cache.begin(); it != c->cache.end(); ++it)
      if (it->second->refs == 0 && (victim == c->cache.end() || it->second->last_use < victim->second->last_use))
        victim = it;
    if (victim == c->cache.end()) return false;
    fntrs_locator_t* L = victim->second;
    c->cache.erase(victim);
    free_locator(c, L);
  }
  return true;
}

static int build_locator(fntrs_ctx* c, fntrs_locator_t* L, hipStream_t s) {
  const uint32_t n = L->n, k = L->k;
  const int logn = L->logn, logk = L->logk;
  const size_t M = (k < n) ? (size_t)1 << L->logm : 0;
  // device layout: pos[k] wfull[n] ridx[n] ahat_br[M] ahat_s[M] A[k+1] w[k] ahat[M]
  //                | scratch: t0[k] t1[k] spec[k] vals[n]
  const size_t state = k + 2ull * n + 2 * M + (k + 1) + k + M;
  const size_t scratch = (k < n) ? 3ull * k + n : 0;
  L->bytes = (state + scratch) * 4;
  if (!make_room(c, L->bytes))
    return fail(c, FNTRS_E_NOMEM, "locator of %zu bytes exceeds the context cap (%zu used of %zu)", L->bytes,
                c->used, c->cap);
  hipError_t e = hipMalloc((void**)&L->mem, L->bytes);
  if (e != hipSuccess) {
    L->mem = nullptr;
    return fail(c, FNTRS_E_NOMEM, "hipMalloc(%zu) for locator failed: %s", L->bytes, hipGetErrorString(e));
  }
  c->used += L->bytes;
  uint32_t* p = L->mem;
  L->pos = p; p += k;
  L->wfull = p; p += n;
  L->ridx = p; p += n;
  L->ahat_br = p; p += M;
  L->ahat_s = p; p += M;
  L->A = p; p += k + 1;
  L->w = p; p += k;
  L->ahat = p; p += M;
  uint32_t* t0 = p; p += (k < n) ? k : 0;
  uint32_t* t1 = p; p += (k < n) ? k : 0;
  uint32_t* spec = p; p += (k < n) ? k : 0;
  uint32_t* vals = p;

  HIP_TRY(c, hipMemcpyAsync(L->pos, L->positions.data(), k * 4ull, hipMemcpyHostToDevice, s));
  if (k == n) {
    // Nothing erased: the decoder is the inverse FNT_n with factor n^-1.
    const uint32_t ninv = 65537u - (65536u >> logn);
    hipLaunchKernelGGL(k_loc_identity, dim3((n + 255) / 256), dim3(256), 0, s, L->wfull, L->ridx, n, ninv);
    // A = x^n - 1 for export
    hipLaunchKernelGGL(k_loc_fill, dim3((k + 256) / 256), dim3(256), 0, s, L->A, k + 1, 0u);
    hipLaunchKernelGGL(k_loc_fill, dim3(1), dim3(1), 0, s, L->A, 1u, 65536u);
    hipLaunchKernelGGL(k_loc_fill, dim3(1), dim3(1), 0, s, L->A + k, 1u, 1u);
    HIP_TRY(c, hipGetLastError());
  } else {
    // Step 1: product tree.  Leaves of G points, then FNT products up to degree k.
    const int G = (int)std::min<uint32_t>(k, 64);
    hipLaunchKernelGGL(k_loc_leaves, dim3(k / G), dim3(64), 0, s, L->pos, logn, G, c->tw, t0);
    HIP_TRY(c, hipGetLastError());
    uint32_t* cur = t0;
    uint32_t* nxt = t1;
    for (uint32_t d = G; d < k; d *= 2) {
      const size_t lds = 2ull * d * 4;
      (void)set_lds_attr((const void*)k_loc_mul_level, lds);
      const int nt = (int)std::min<uint32_t>(1024, std::max<uint32_t>(64, d / 2));
      hipLaunchKernelGGL(k_loc_mul_level, dim3(k / (2 * d)), dim3(nt), lds, s, cur, ilog2(d), c->tw, spec, nxt);
      HIP_TRY(c, hipGetLastError());
      std::swap(cur, nxt);
    }
    // cur holds a_0..a_(k-1); A = x^k + ...
    HIP_TRY(c, hipMemcpyAsync(L->A, cur, k * 4ull, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_loc_fill, dim3(1), dim3(1), 0, s, L->A + k, 1u, 1u);
    HIP_TRY(c, hipGetLastError());
    // Step 2: A'.
    hipLaunchKernelGGL(k_loc_derivative, dim3((k + 255) / 256), dim3(256), 0, s, cur, k, spec);
    HIP_TRY(c, hipGetLastError());
    // Step 3: A' at every n-th root (n/k twisted FNT_k), then the weights.
    const size_t ldsk = (size_t)k * 4;
    (void)set_lds_attr((const void*)k_loc_eval, ldsk);
    const int ntk = (int)std::min<uint32_t>(1024, std::max<uint32_t>(64, k / 4));
    hipLaunchKernelGGL(k_loc_eval, dim3(n / k), dim3(ntk), ldsk, s, spec, logk, logn, c->tw, vals);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(k_loc_fill, dim3((n + 255) / 256), dim3(256), 0, s, L->wfull, n, 0u);
    hipLaunchKernelGGL(k_loc_weights, dim3((k + 255) / 256), dim3(256), 0, s, L->pos, vals, k, logn, c->tw, L->w,
                       L->wfull, L->ridx);
    HIP_TRY(c, hipGetLastError());
    // FNT_M of (a_0..a_(k-1), 0..0): M/k twisted FNT_k; then the decoder's
    // copy, bit-reversed and scaled by M^-1.
    hipLaunchKernelGGL(k_loc_eval, dim3((uint32_t)(M / k)), dim3(ntk), ldsk, s, cur, logk, L->logm, c->tw, L->ahat);
    HIP_TRY(c, hipGetLastError());
    hipLaunchKernelGGL(k_loc_ahat, dim3((uint32_t)((M + 255) / 256)), dim3(256), 0, s, L->ahat, L->logm, L->ahat_br,
                       L->ahat_s);
    HIP_TRY(c, hipGetLastError());
  }
  HIP_TRY(c, hipEventCreateWithFlags(&L->ready, hipEventDisableTiming));
  HIP_TRY(c, hipEventRecord(L->ready, s));
  return FNTRS_OK;
}

hipError_t launch_copy(const uint32_t* src, size_t stride_src, uint32_t* dst, size_t stride_dst, uint32_t lanes,
                       uint32_t batch, hipStream_t s) {
  const uint64_t total = (uint64_t)lanes * batch;
  hipLaunchKernelGGL(k_copy_rows, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, src, (uint64_t)stride_src,
                     dst, (uint64_t)stride_dst, lanes, batch, (const uint32_t*)nullptr);
  return hipGetLastError();
}

int locator_acquire(fntrs_ctx* c, uint32_t n, uint32_t k, const uint32_t* positions, uint32_t npos,
                    hipStream_t stream, fntrs_locator_t** out) {
  if (!out) return fail(c, FNTRS_E_INVAL, "null out");
  *out = nullptr;
  if (!is_pow2(n) || n > 65536) return fail(c, FNTRS_E_INVAL, "n=%u must be a power of two in [1, 65536]", n);
  if (k < 1 || k > n) return fail(c, FNTRS_E_INVAL, "k=%u must satisfy 1 <= k <= n=%u", k, n);
  if (!positions) return fail(c, FNTRS_E_INVAL, "null positions");
  if (npos < k) return fail(c, FNTRS_E_TOOFEW, "%u positions received, k=%u needed", npos, k);
  for (uint32_t i = 0; i < k; ++i) {
    if (positions[i] >= n) return fail(c, FNTRS_E_POSITIONS, "position %u at index %u is >= n=%u", positions[i], i, n);
    if (i && positions[i] <= positions[i - 1])
      return fail(c, FNTRS_E_POSITIONS, "positions must be strictly ascending (index %u)", i);
  }
  if (!is_pow2(k)) return fail(c, FNTRS_E_UNSUPPORTED, "decoding needs k a power of two, got %u", k);
  const uint64_t key = hash_positions(n, k, positions);
  auto range = c->cache.equal_range(key);
  for (auto it = range.first; it != range.second; ++it) {
    fntrs_locator_t* L = it->second;
    if (L->n == n && L->k == k && std::equal(L->positions.begin(), L->positions.end(), positions)) {
      L->refs++;
      L->last_use = ++c->tick;
      *out = L;
      return FNTRS_OK;
    }
  }
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
  DeviceGuard g(c->device);
  auto* L = new fntrs_locator_t();
  L->n = n; L->k = k; L->logn = ilog2(n); L->logk = ilog2(k);
  L->logm = std::max(L->logk + 1, L->logn - 1);   // low-product length M >= 2k, M >= n/2
  L->positions.assign(positions, positions + k);
  L->key = key;
  int rc = build_locator(c, L, stream);
  if (rc) {
    free_locator(c, L);
    return rc;
  }
  L->refs = 1;
  L->last_use = ++c->tick;
  c->cache.emplace(key, L);
  *out = L;
  return FNTRS_OK;
}

// Default kernel configuration per transform size, then the FNTRS_TILES
// override "e12=8x512,d13=4x1024,...".
void set_default_configs(fntrs_ctx* c) {
  for (int L = 1; L <= 15; ++L) {
    c->enc_cfg[L] = ct_variants(L).enc[0];
    c->dec_cfg[L] = ct_variants(L).dec[0];
  }
  // FNTRS_TILES="e12=8x512,d13=4x1024,...": override the configuration per size
  if (const char* t = getenv("FNTRS_TILES")) {
    std::string spec(t);
    size_t pos = 0;
    while (pos < spec.size()) {
      size_t end = spec.find(',', pos);
      if (end == std::string::npos) end = spec.size();
      const std::string item = spec.substr(pos, end - pos);
      int L = 0, T = 0, NT = 512;
      char kind = 0;
      if (sscanf(item.c_str(), "%c%d=%dx%d", &kind, &L, &T, &NT) >= 3 && L >= 1 && L <= 15) {
        if (kind == 'e') c->enc_cfg[L] = CtCfg{T, NT};
        if (kind == 'd') c->dec_cfg[L] = CtCfg{T, NT};
      }
      pos = end + 1;
    }
  }
}

}  // namespace fntrs

using namespace fntrs;

extern "C" {

const char* fntrs_version(void) { return "fntrs 0.1 (gfx950)"; }

int fntrs_create(int device, size_t cap, fntrs_ctx** out) {
  if (!out) return FNTRS_E_INVAL;
  *out = nullptr;
  if (device == FNTRS_HOST_ONLY) {
    auto* c = new fntrs_ctx();
    c->device = FNTRS_HOST_ONLY;
    c->cap = cap ? cap : kDefaultCap;
    c->lds_max = 163840;
    set_default_configs(c);
    *out = c;
    return FNTRS_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return FNTRS_E_DEVICE;
  if (device < 0 || device >= ndev) return FNTRS_E_INVAL;
  auto* c = new fntrs_ctx();
  c->device = device;
  c->cap = cap ? cap : kDefaultCap;
  DeviceGuard g(device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete c; return FNTRS_E_DEVICE; }
  c->lds_max = prop.sharedMemPerBlock;
  c->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  set_default_configs(c);
  // twiddle tables: tw[e] = 3^e and twi[e] = 3^-e = 3^(65536-e), e < 65536
  std::vector<uint32_t> h(2 * 65536);
  uint64_t x = 1;
  for (int e = 0; e < 65536; ++e) { h[e] = (uint32_t)x; x = x * 3 % 65537; }
  for (int e = 0; e < 65536; ++e) h[65536 + e] = h[(65536 - e) & 0xFFFF];
  if (hipMalloc((void**)&c->tw, 2 * 65536 * 4) != hipSuccess) { delete c; return FNTRS_E_NOMEM; }
  c->twi = c->tw + 65536;
  c->used += 2 * 65536 * 4;
  if (hipMemcpy(c->tw, h.data(), 2 * 65536 * 4, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c->tw);
    delete c;
    return FNTRS_E_DEVICE;
  }
  *out = c;
  return FNTRS_OK;
}

void fntrs_destroy(fntrs_ctx* c) {
  if (!c) return;
  if (c->device == FNTRS_HOST_ONLY) { delete c; return; }
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : c->cache) free_locator(c, kv.second);
  c->cache.clear();
  for (int b = 0; b < fntrs_ctx::kSide; ++b) {
    if (c->side[b]) (void)hipStreamDestroy(c->side[b]);
    if (c->join[b]) (void)hipEventDestroy(c->join[b]);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->tw) (void)hipFree(c->tw);
  delete c;
}

const char* fntrs_last_error(const fntrs_ctx* c) { return c ? c->err.c_str() : "null context"; }

int fntrs_encode(fntrs_ctx* c, uint32_t n, uint32_t k, uint32_t lanes, const uint32_t* src, size_t ld_src,
                 size_t stride_src, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch, uint32_t flags,
                 void* stream) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (int rc = check_encode(c, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, flags)) return rc;
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  if (flags & FNTRS_FLAG_VALIDATE) {
    int rc = validate_range(c, src, batch, stride_src, k, ld_src, lanes, s);
    if (rc) return rc;
  }
  if (n == 1) {  // k = 1: e_0 = s_0
    HIP_TRY(c, launch_copy(src, stride_src, dst, stride_dst, lanes, batch, s));
    return FNTRS_OK;
  }
  EncodeArgs a;
  a.src = src; a.ld_src = ld_src; a.stride_src = stride_src;
  a.dst = dst; a.ld_dst = ld_dst; a.stride_dst = stride_dst;
  a.tw = c->tw; a.twi = c->twi;
  a.n = n; a.k = k; a.lanes = lanes;
  a.logn = ilog2(n);
  a.logK = std::max(1, ilog2(k));        // transform size K: smallest power of two >= k, at least 2
  if (a.logK == 16) {
    // K = n = 65536: four-step transform through a scratch buffer
    FourStepArgs f{};
    f.in = src; f.ld_in = ld_src; f.stride_in = stride_src;
    f.out = dst; f.ld_out = ld_dst; f.stride_out = stride_dst;
    f.tw = c->tw; f.twi = c->twi;
    f.n = n; f.k = k; f.M = n; f.lanes = lanes; f.logn = 16; f.logm = 16;
    f.tiles = (lanes + kFourStepTile - 1) / kFourStepTile;
    const uint64_t lds = (uint64_t)f.tiles * kFourStepTile;
    f.vec = aligned16(src, ld_src, stride_src) && aligned16(dst, ld_dst, stride_dst);
    uint32_t* sa = nullptr;
    const size_t bytes = (size_t)batch * n * lds * 4;
    hipError_t e = hipMallocAsync((void**)&sa, bytes, s);
    if (e != hipSuccess) return fail(c, FNTRS_E_NOMEM, "scratch of %zu bytes: %s", bytes, hipGetErrorString(e));
    e = fourstep_encode(f, batch, sa, lds, s);
    (void)hipFreeAsync(sa, s);
    HIP_TRY(c, e);
    return FNTRS_OK;
  }
  const CtCfg cfg = c->enc_cfg[a.logK];
  a.vec = aligned16(src, ld_src, stride_src) && aligned16(dst, ld_dst, stride_dst);
  a.tiles = (lanes + cfg.T - 1) / cfg.T;
  a.cosets = n >> a.logK;
  const uint64_t blocks = (uint64_t)a.tiles * a.cosets * batch;
  if (blocks > 0x7fffffffull) return fail(c, FNTRS_E_INVAL, "grid too large");
  HIP_TRY(c, ct_tables().enc[a.logK](cfg, a, (uint32_t)blocks, s));
  return FNTRS_OK;
}

int fntrs_locator(fntrs_ctx* c, uint32_t n, uint32_t k, const uint32_t* positions, uint32_t npos, void* stream,
                  fntrs_locator_t** out) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  return locator_acquire(c, n, k, positions, npos, (hipStream_t)stream, out);
}

int fntrs_locator_release(fntrs_ctx* c, fntrs_locator_t* L) {
  if (!c || !L) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (L->refs <= 0) return fail(c, FNTRS_E_INVAL, "locator released more often than acquired");
  L->refs--;
  return FNTRS_OK;
}

int fntrs_locator_export(fntrs_ctx* c, const fntrs_locator_t* L, uint32_t* A, uint32_t* w, uint32_t* ahat) {
  if (!c || !L) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context");
  DeviceGuard g(c->device);
  HIP_TRY(c, hipEventSynchronize(L->ready));
  if (A) HIP_TRY(c, hipMemcpy(A, L->A, (L->k + 1) * 4ull, hipMemcpyDeviceToHost));
  if (w) HIP_TRY(c, hipMemcpy(w, L->w, L->k * 4ull, hipMemcpyDeviceToHost));
  if (ahat && L->k != L->n) {
    // FNT_2k values are the FNT_M values at multiples of M/2k
    const size_t M = (size_t)1 << L->logm, step = M / (2ull * L->k);
    std::vector<uint32_t> h(M);
    HIP_TRY(c, hipMemcpy(h.data(), L->ahat, M * 4, hipMemcpyDeviceToHost));
    for (size_t m = 0; m < 2ull * L->k; ++m) ahat[m] = h[m * step];
  }
  return FNTRS_OK;
}

int fntrs_decode(fntrs_ctx* c, const fntrs_locator_t* L, uint32_t lanes, uint32_t flags, const uint32_t* recv,
                 size_t ld_recv, size_t stride_recv, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
                 void* stream) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (int rc = check_decode(c, L, lanes, flags, recv, ld_recv, stride_recv, dst, ld_dst, stride_dst, batch)) return rc;
  const bool full = flags & FNTRS_RECV_FULL;
  const uint32_t n = L->n, k = L->k;
  const uint32_t rrows = full ? n : k;
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  if (flags & FNTRS_FLAG_VALIDATE) {
    int rc = validate_range(c, recv, batch, stride_recv, rrows, ld_recv, lanes, s);
    if (rc) return rc;
  }
  HIP_TRY(c, hipStreamWaitEvent(s, L->ready, 0));
  if (n == 1) {  // k = n = 1: s_0 = e_0
    HIP_TRY(c, launch_copy(recv, stride_recv, dst, stride_dst, lanes, batch, s));
    return FNTRS_OK;
  }
  if (L->logn == 16) {
    FourStepArgs f{};
    f.in = recv; f.ld_in = ld_recv; f.stride_in = stride_recv;
    f.out = dst; f.ld_out = ld_dst; f.stride_out = stride_dst;
    f.tw = c->tw; f.twi = c->twi; f.wfull = L->wfull; f.ridx = L->ridx; f.ahat = L->ahat_s;
    f.n = n; f.k = k; f.lanes = lanes; f.logn = 16;
    f.logm = (k == n) ? 16 : L->logm;
    f.M = 1u << f.logm;
    f.full = full ? 1u : 0u;
    f.tiles = (lanes + kFourStepTile - 1) / kFourStepTile;
    const uint64_t lds = (uint64_t)f.tiles * kFourStepTile;
    f.vec = aligned16(recv, ld_recv, stride_recv) && aligned16(dst, ld_dst, stride_dst);
    uint32_t* sa = nullptr;
    const size_t bytes = (size_t)batch * (n + f.M) * lds * 4;
    hipError_t e = hipMallocAsync((void**)&sa, bytes, s);
    if (e != hipSuccess) return fail(c, FNTRS_E_NOMEM, "scratch of %zu bytes: %s", bytes, hipGetErrorString(e));
    e = fourstep_decode(f, batch, sa, sa + (size_t)batch * n * lds, lds, s);
    (void)hipFreeAsync(sa, s);
    HIP_TRY(c, e);
    return FNTRS_OK;
  }
  DecodeArgs a;
  a.recv = recv; a.ld_recv = ld_recv; a.stride_recv = stride_recv;
  a.dst = dst; a.ld_dst = ld_dst; a.stride_dst = stride_dst;
  a.tw = c->tw; a.twi = c->twi; a.wfull = L->wfull; a.ridx = L->ridx; a.ahat_br = L->ahat_br;
  a.n = n; a.k = k; a.lanes = lanes; a.logn = L->logn; a.logk = L->logk;
  a.full = full ? 1u : 0u;
  const int D = (k == n) ? -1 : L->logn - L->logm;
  const CtCfg cfg = c->dec_cfg[L->logn];
  a.vec = aligned16(recv, ld_recv, stride_recv) && aligned16(dst, ld_dst, stride_dst);
  a.tiles = (lanes + cfg.T - 1) / cfg.T;
  const uint64_t blocks = (uint64_t)a.tiles * batch;
  if (blocks > 0x7fffffffull) return fail(c, FNTRS_E_INVAL, "grid too large");
  HIP_TRY(c, ct_tables().dec[L->logn](cfg, D, a, (uint32_t)blocks, s));
  return FNTRS_OK;
}

}  // extern "C"
