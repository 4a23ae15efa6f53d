// libfntrs: host side of the C ABI declared in include/fntrs.h.
//
// Validation happens here, synchronously, before anything is enqueued; the
// coding work itself runs in the compile-time kernels (ct_kernels.hpp, one
// translation unit per transform size) and the locator kernels
// (locator_kernels.hpp).  The batched path (jobs, graphs, autotuning) is in
// submit.hip.
#include <set>

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
  static const CtEncCosLaunch enc_cos[16] = {
      nullptr,              ct_enc_cos_launch_1,  ct_enc_cos_launch_2,  ct_enc_cos_launch_3,
      ct_enc_cos_launch_4,  ct_enc_cos_launch_5,  ct_enc_cos_launch_6,  ct_enc_cos_launch_7,
      ct_enc_cos_launch_8,  ct_enc_cos_launch_9,  ct_enc_cos_launch_10, ct_enc_cos_launch_11,
      ct_enc_cos_launch_12, ct_enc_cos_launch_13, ct_enc_cos_launch_14, ct_enc_cos_launch_15};
  static const CtDecPipeLaunch dec_pipe[16] = {
      nullptr,               ct_dec_pipe_launch_1,  ct_dec_pipe_launch_2,  ct_dec_pipe_launch_3,
      ct_dec_pipe_launch_4,  ct_dec_pipe_launch_5,  ct_dec_pipe_launch_6,  ct_dec_pipe_launch_7,
      ct_dec_pipe_launch_8,  ct_dec_pipe_launch_9,  ct_dec_pipe_launch_10, ct_dec_pipe_launch_11,
      ct_dec_pipe_launch_12, ct_dec_pipe_launch_13, ct_dec_pipe_launch_14, ct_dec_pipe_launch_15};
  static const CtEncCosTabLaunch enc_cos_tab[16] = {
      nullptr,                  ct_enc_cos_tab_launch_1,  ct_enc_cos_tab_launch_2,  ct_enc_cos_tab_launch_3,
      ct_enc_cos_tab_launch_4,  ct_enc_cos_tab_launch_5,  ct_enc_cos_tab_launch_6,  ct_enc_cos_tab_launch_7,
      ct_enc_cos_tab_launch_8,  ct_enc_cos_tab_launch_9,  ct_enc_cos_tab_launch_10, ct_enc_cos_tab_launch_11,
      ct_enc_cos_tab_launch_12, ct_enc_cos_tab_launch_13, ct_enc_cos_tab_launch_14, ct_enc_cos_tab_launch_15};
  static const CtTables t{enc, dec, enc_tab, dec_tab, enc_cos, dec_pipe, occ, enc_cos_tab};
  return t;
}

void lds_attr_once(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::set<std::tuple<const void*, int, size_t>> done;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lk(mu);
  if (done.insert({fn, dev, bytes}).second)
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// A pinned staging slot of at least `bytes`, idle (its last use complete);
// the caller fills it, enqueues what reads it, then records slot->ev on that
// stream and sets slot->pending.
int stage_slot(fntrs_ctx* c, size_t bytes, fntrs_ctx::StageSlot*& out) {
  constexpr size_t kMaxSlots = 32;
  fntrs_ctx::StageSlot* slot = nullptr;
  for (auto& q : c->stage) {   // an idle slot that is large enough
    if (q.bytes >= bytes && (!q.pending || hipEventQuery(q.ev) == hipSuccess)) { slot = &q; break; }
  }
  if (!slot) {                 // else an idle slot to grow, or a new one
    for (auto& q : c->stage)
      if (!q.pending || hipEventQuery(q.ev) == hipSuccess) { slot = &q; break; }
    if (!slot && c->stage.size() < kMaxSlots) {
      c->stage.emplace_back();
      slot = &c->stage.back();
      HIP_TRY(c, hipEventCreateWithFlags(&slot->ev, hipEventDisableTiming));
    }
    if (!slot) {               // all busy: wait for the first
      slot = &c->stage.front();
      HIP_TRY(c, hipEventSynchronize(slot->ev));
    }
    if (slot->bytes < bytes) {
      if (slot->p) HIP_TRY(c, hipHostFree(slot->p));
      slot->p = nullptr;
      slot->bytes = 0;
      size_t sz = 65536;
      while (sz < bytes) sz <<= 1;
      HIP_TRY(c, hipHostMalloc(&slot->p, sz, hipHostMallocDefault));
      slot->bytes = sz;
    }
  }
  out = slot;
  return FNTRS_OK;
}

int upload_async(fntrs_ctx* c, void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return FNTRS_OK;
  fntrs_ctx::StageSlot* slot = nullptr;
  if (int rc = stage_slot(c, bytes, slot)) return rc;
  std::memcpy(slot->p, src, bytes);
  HIP_TRY(c, hipMemcpyAsync(dst, slot->p, bytes, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipEventRecord(slot->ev, s));
  slot->pending = true;
  return FNTRS_OK;
}

void stage_release(fntrs_ctx* c) {
  for (auto& q : c->stage) {
    if (q.p) (void)hipHostFree(q.p);
    if (q.ev) (void)hipEventDestroy(q.ev);
  }
  c->stage.clear();
  for (auto& q : c->dev_slots) {
    if (q.p) (void)hipFree(q.p);
    if (q.ev) (void)hipEventDestroy(q.ev);
  }
  c->dev_slots.clear();
}

int dev_slot_acquire(fntrs_ctx* c, size_t bytes, fntrs_ctx::DevSlot*& out) {
  constexpr size_t kMaxSlots = 8;
  out = nullptr;
  auto idle = [](fntrs_ctx::DevSlot& q) {
    return !q.busy && (!q.pending || hipEventQuery(q.ev) == hipSuccess);
  };
  for (auto& q : c->dev_slots)   // the smallest idle slot that fits
    if (q.bytes >= bytes && idle(q) && (!out || q.bytes < out->bytes)) out = &q;
  if (out) {
    out->busy = true;
    return FNTRS_OK;
  }
  fntrs_ctx::DevSlot* slot = nullptr;
  if (c->dev_slots.size() < kMaxSlots) {
    c->dev_slots.emplace_back();
    slot = &c->dev_slots.back();
    HIP_TRY(c, hipEventCreateWithFlags(&slot->ev, hipEventDisableTiming));
  } else {                       // replace the smallest slot no call holds, once it is idle
    for (auto& q : c->dev_slots)
      if (!q.busy && (!slot || q.bytes < slot->bytes)) slot = &q;
    if (!slot) return fail(c, FNTRS_E_DEVICE, "every device table slot is held");
    if (slot->pending) HIP_TRY(c, hipEventSynchronize(slot->ev));
    HIP_TRY(c, hipFree(slot->p));
    slot->p = nullptr;
    slot->bytes = 0;
  }
  size_t sz = size_t(1) << 20;
  while (sz < bytes) sz <<= 1;
  if (hipMalloc((void**)&slot->p, sz) != hipSuccess) {
    slot->p = nullptr;
    return fail(c, FNTRS_E_NOMEM, "device table buffer of %zu bytes", sz);
  }
  slot->bytes = sz;
  slot->pending = false;
  slot->busy = true;
  out = slot;
  return FNTRS_OK;
}

int dev_slot_done(fntrs_ctx* c, fntrs_ctx::DevSlot* slot, hipStream_t s) {
  slot->busy = false;
  if (hipEventRecord(slot->ev, s) != hipSuccess) {
    (void)hipStreamSynchronize(s);   // no event: wait here rather than reuse early
    slot->pending = false;
    return fail(c, FNTRS_E_DEVICE, "event record after a device table slot");
  }
  slot->pending = true;
  return FNTRS_OK;
}

int scratch_acquire(fntrs_ctx* c, size_t bytes, hipStream_t s, Scratch& out) {
  out = Scratch{};
  if (bytes == 0) return FNTRS_OK;
  if (bytes <= kDevSlotMax) {
    fntrs_ctx::DevSlot* d = nullptr;
    if (int rc = dev_slot_acquire(c, bytes, d)) return rc;
    out = Scratch{d->p, 1, d};
    return FNTRS_OK;
  }
  using Blk = fntrs_ctx::WsBlock;
  auto idle = [](Blk& b) { return !b.busy && (!b.pending || hipEventQuery(b.ev) == hipSuccess); };
  Blk* best = nullptr;
  for (auto& b : c->ws)   // the smallest idle block that fits
    if (b.bytes >= bytes && idle(b) && (!best || b.bytes < best->bytes)) best = &b;
  if (!best) {            // a new block, if the cap allows
    constexpr size_t kGrain = size_t(256) << 20;
    const size_t want = (bytes + kGrain - 1) / kGrain * kGrain;
    uint8_t* p = nullptr;
    if (c->ws_held + want <= c->cap && hipMalloc((void**)&p, want) == hipSuccess) {
      hipEvent_t ev = nullptr;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(p);
        return fail(c, FNTRS_E_DEVICE, "event for a workspace block");
      }
      c->ws.emplace_back();
      best = &c->ws.back();
      best->p = p;
      best->bytes = want;
      best->ev = ev;
      c->ws_held += want;
    }
  }
  if (!best) {            // a block still in use on some stream, after that use
    for (auto& b : c->ws)
      if (!b.busy && b.bytes >= bytes && (!best || b.bytes < best->bytes)) best = &b;
    if (best && best->pending) HIP_TRY(c, hipStreamWaitEvent(s, best->ev, 0));
  }
  if (best) {
    best->busy = true;
    out = Scratch{best->p, 2, best};
    return FNTRS_OK;
  }
  uint8_t* p = nullptr;   // nothing fits under the cap: stream-ordered memory
  const hipError_t e = hipMallocAsync((void**)&p, bytes, s);
  if (e != hipSuccess) return fail(c, FNTRS_E_NOMEM, "scratch of %zu bytes: %s", bytes, hipGetErrorString(e));
  out = Scratch{p, 3, nullptr};
  return FNTRS_OK;
}

void scratch_release(fntrs_ctx* c, Scratch& sc, hipStream_t s) {
  if (sc.kind == 1) {
    (void)dev_slot_done(c, static_cast<fntrs_ctx::DevSlot*>(sc.ref), s);
  } else if (sc.kind == 2) {
    auto* b = static_cast<fntrs_ctx::WsBlock*>(sc.ref);
    b->pending = hipEventRecord(b->ev, s) == hipSuccess;
    if (!b->pending) (void)hipStreamSynchronize(s);   // no event: wait here rather than reuse early
    b->busy = false;
  } else if (sc.kind == 3) {
    (void)hipFreeAsync(sc.p, s);
  }
  sc = Scratch{};
}

void workspace_release(fntrs_ctx* c) {
  for (auto& b : c->ws) {
    if (b.p) (void)hipFree(b.p);
    if (b.ev) (void)hipEventDestroy(b.ev);
  }
  c->ws.clear();
  c->ws_held = 0;
}

// The configuration of one single call: the size's configuration, or its
// narrow tile when the call would otherwise give fewer work items than half
// the CUs (per = work items per lane tile).
CtCfg call_cfg(const fntrs_ctx* c, CtCfg cfg, int L, uint32_t lanes, uint64_t per) {
  const CtCfg sm = ct_small(L);
  if (sm.T == 0 || sm.T >= cfg.T) return cfg;
  const uint64_t items = (uint64_t)((lanes + cfg.T - 1) / cfg.T) * per;
  return items * 2 < (uint64_t)c->num_cu ? sm : cfg;
}

int kernel_occupancy(fntrs_ctx* c, int op, int L, int D, CtCfg cfg) {
  const auto key = std::make_tuple(op, L, D, cfg.T * 4096 + cfg.NT, cfg.V);
  auto it = c->occ.find(key);
  if (it != c->occ.end()) return it->second;
  const int o = ct_tables().occ[L](cfg, op, D);
  c->occ[key] = o;
  return o;
}

hipError_t launch_ct_encode(fntrs_ctx* c, int L, CtCfg cfg, const EncodeArgs& a, uint64_t items, hipStream_t s) {
  (void)c;
  if (items > 0x7fffffffull) return hipErrorInvalidValue;
  if (a.cosets >= 2) {   // every coset of a lane tile in one workgroup, when the shape allows
    const hipError_t e = ct_tables().enc_cos[L](cfg, a, (uint32_t)(items / a.cosets), s);
    if (e != hipErrorNotSupported) return e;
  }
  return ct_tables().enc[L](cfg, a, (uint32_t)items, s);
}

hipError_t launch_ct_decode(fntrs_ctx* c, int L, CtCfg cfg, int D, const DecodeArgs& a, uint64_t items,
                            hipStream_t s) {
  if (items > 0x7fffffffull) return hipErrorInvalidValue;
  const int occ = kernel_occupancy(c, 2, L, D, cfg);
  if (occ > 0) {
    const JobTable<DecodeArgs> t{nullptr, nullptr, 1, (uint32_t)items};
    const uint32_t grid = (uint32_t)std::min<uint64_t>(items, (uint64_t)occ * c->num_cu);
    return ct_tables().dec_pipe[L](cfg, D, t, a, c->tw, c->twi, grid, s);
  }
  return ct_tables().dec[L](cfg, D, a, (uint32_t)items, s);
}

int check_encode(fntrs_ctx* c, uint32_t n, uint32_t k, uint32_t lanes, const uint32_t* src, size_t ld_src,
                 size_t stride_src, const uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
                 uint32_t flags) {
  if (n < 1 || n > 65536) return fail(c, FNTRS_E_INVAL, "n=%u must lie in [1, 65536]", n);
  if (k < 1 || k > n) return fail(c, FNTRS_E_INVAL, "k=%u must satisfy 1 <= k <= n=%u", k, n);
  if (lanes < 1 || batch < 1) return fail(c, FNTRS_E_INVAL, "lanes=%u and batch=%u must be >= 1", lanes, batch);
  if (!src || !dst) return fail(c, FNTRS_E_INVAL, "null src or dst");
  if (ld_src < lanes || ld_dst < lanes) return fail(c, FNTRS_E_INVAL, "ld_src/ld_dst smaller than lanes");
  if (batch > 1 && (stride_src < (size_t)(k - 1) * ld_src + lanes || stride_dst < (size_t)(n - 1) * ld_dst + lanes))
    return fail(c, FNTRS_E_INVAL, "block strides overlap consecutive blocks");
  if (flags & ~(FNTRS_FLAG_VALIDATE | FNTRS_SYSTEMATIC | FNTRS_DIRECT | FNTRS_TRANSFORM))
    return fail(c, FNTRS_E_INVAL, "unknown flags 0x%x", flags);
  if ((flags & FNTRS_DIRECT) && (flags & FNTRS_TRANSFORM))
    return fail(c, FNTRS_E_INVAL, "FNTRS_DIRECT and FNTRS_TRANSFORM exclude each other");
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
  if (flags & ~(FNTRS_RECV_FULL | FNTRS_FLAG_VALIDATE | FNTRS_SYSTEMATIC | FNTRS_DIRECT | FNTRS_TRANSFORM))
    return fail(c, FNTRS_E_INVAL, "unknown flags 0x%x", flags);
  if ((flags & FNTRS_DIRECT) && (flags & FNTRS_TRANSFORM))
    return fail(c, FNTRS_E_INVAL, "FNTRS_DIRECT and FNTRS_TRANSFORM exclude each other");
  const bool full = flags & FNTRS_RECV_FULL;
  const uint32_t k = L->k;
  const uint32_t rrows = full ? L->nrows : k;
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
  lds_attr_once(fn, bytes);
  return hipSuccess;
}

// One launch of a locator stage on the one-lane ct kernels (transform size
// 2^L).
template <int L>
void launch_level_ct(uint32_t grid, const LocDesc* D, const uint32_t* start, uint32_t count, int lev,
                     const uint32_t* tw, const uint32_t* twi, hipStream_t s) {
  constexpr size_t lds = LocGeo<L>::LDS_BYTES;
  (void)set_lds_attr((const void*)k_locb_level_ct<L>, lds);
  hipLaunchKernelGGL(k_locb_level_ct<L>, dim3(grid), dim3(loc_nt<L>()), lds, s, D, start, count, lev, tw, twi);
}
template <int L>
void launch_eval_ct(uint32_t grid, const LocDesc* D, const uint32_t* start, uint32_t count, const uint32_t* tw,
                    const uint32_t* twi, hipStream_t s) {
  constexpr size_t lds = LocGeo<L>::LDS_BYTES;
  (void)set_lds_attr((const void*)k_locb_eval_ct<L>, lds);
  hipLaunchKernelGGL(k_locb_eval_ct<L>, dim3(grid), dim3(loc_nt<L>()), lds, s, D, start, count, tw, twi);
}
// false when L has no one-lane ct kernel (the caller uses the radix-4 one)
bool level_ct(int L, uint32_t grid, const LocDesc* D, const uint32_t* start, uint32_t count, int lev,
              const uint32_t* tw, const uint32_t* twi, hipStream_t s) {
  if (L < kLocLevelCtMin) return false;
  switch (L) {
    case 12: launch_level_ct<12>(grid, D, start, count, lev, tw, twi, s); return true;
    case 13: launch_level_ct<13>(grid, D, start, count, lev, tw, twi, s); return true;
    case 14: launch_level_ct<14>(grid, D, start, count, lev, tw, twi, s); return true;
    case 15: launch_level_ct<15>(grid, D, start, count, lev, tw, twi, s); return true;
    default: return false;
  }
}
bool eval_ct(int L, uint32_t grid, const LocDesc* D, const uint32_t* start, uint32_t count, const uint32_t* tw,
             const uint32_t* twi, hipStream_t s) {
  if (L < kLocEvalCtMin) return false;
  switch (L) {
    case 11: launch_eval_ct<11>(grid, D, start, count, tw, twi, s); return true;
    case 12: launch_eval_ct<12>(grid, D, start, count, tw, twi, s); return true;
    case 13: launch_eval_ct<13>(grid, D, start, count, tw, twi, s); return true;
    case 14: launch_eval_ct<14>(grid, D, start, count, tw, twi, s); return true;
    case 15: launch_eval_ct<15>(grid, D, start, count, tw, twi, s); return true;
    default: return false;
  }
}

// FNT_n (n = 2^14 .. 2^16) of `lanes` <= kFourStepTile vectors stored
// [row][lanes]: k <= n rows at src, zero-padded to n, natural order in and
// out, on the four-step kernels -- hundreds of workgroups where a one-lane
// transform of the lane-tile kernels runs in one or two.
// `scr` holds n * kFourStepTile words (kFnOneScratchWords covers any n).
constexpr size_t kFnOneScratchWords = size_t(65536) * kFourStepTile;
// Lanes (times blocks) from which a single decode call lays out its first
// pass's (weight, row) pairs (k_dec_pairs) before the transform kernel.
constexpr uint64_t kDecPairsMinLanes = 4096;
int fnt_lanes(fntrs_ctx* c, uint32_t n, uint32_t k, uint32_t lanes, const uint32_t* src, uint32_t* dst, uint32_t* scr,
              hipStream_t s) {
  FourStepArgs f{};
  f.in = src; f.ld_in = lanes; f.stride_in = (size_t)k * lanes;
  f.out = dst; f.ld_out = lanes; f.stride_out = (size_t)n * lanes;
  f.tw = c->tw; f.twi = c->twi;
  f.n = n; f.k = k; f.M = n; f.lanes = lanes; f.logn = ilog2(n); f.logm = f.logn;
  f.tiles = 1;
  HIP_TRY(c, fourstep_encode(f, 1, scr, kFourStepTile, s));
  return FNTRS_OK;
}
int fnt_one(fntrs_ctx* c, uint32_t n, uint32_t k, const uint32_t* src, uint32_t* dst, uint32_t* scr, hipStream_t s) {
  return fnt_lanes(c, n, k, 1, src, dst, scr, s);
}

// Top product-tree level of one pattern (one pair, 2d = the tree's points,
// 2^14 or 2^15) through fnt_one: spec and vals (>= 2d words each, unused
// until the derivative and the evaluation) hold the transforms.
int top_level_fourstep(fntrs_ctx* c, const LocDesc& d, int lev, uint32_t half, uint32_t* scr, hipStream_t s) {
  const uint32_t* in = (lev & 1) ? d.t1 : d.t0;
  uint32_t* out = (lev & 1) ? d.t0 : d.t1;
  const uint32_t n2 = 2 * half;
  if (int rc = fnt_one(c, n2, half, in, d.spec, scr, s)) return rc;          // a_lo
  if (int rc = fnt_one(c, n2, half, in + half, d.vals, scr, s)) return rc;   // b_lo
  hipLaunchKernelGGL(k_loc_mul, dim3((n2 + 255) / 256), dim3(256), 0, s, d.spec, (const uint32_t*)d.vals, n2);
  HIP_TRY(c, hipGetLastError());
  if (int rc = fnt_one(c, n2, n2, d.spec, d.vals, scr, s)) return rc;        // the product, at negated indices
  uint64_t inv = 1, b = n2 % 65537u;                                    // (2d)^-1 = (2d)^65535
  for (uint32_t e = 65535; e; e >>= 1, b = b * b % 65537u)
    if (e & 1u) inv = inv * b % 65537u;
  hipLaunchKernelGGL(k_loc_combine, dim3((n2 + 255) / 256), dim3(256), 0, s, (const uint32_t*)d.vals, in, in + half,
                     out, half, (uint32_t)inv);
  HIP_TRY(c, hipGetLastError());
  return FNTRS_OK;
}

// Logarithmic locator (k_conv_*) for one pattern of n >= 2^kConvMinLog
// positions: a fixed number of launches whatever k, where the product tree
// takes one dependent launch per level, each with few workgroups near the top.
constexpr int kConvMinLog = 12;

// FNT_n of `lanes` vectors stored [n][lanes] (k = n): the four-step kernels
// from 2^14 points (scr: kFnOneScratchWords), the encoder below.
int conv_fnt(fntrs_ctx* c, uint32_t n, uint32_t lanes, const uint32_t* src, uint32_t* dst, uint32_t* scr,
             hipStream_t s) {
  if (n >= (1u << kFourStepMinLog)) return fnt_lanes(c, n, n, lanes, src, dst, scr, s);
  return encode_run(c, n, n, lanes, src, lanes, (size_t)n * lanes, dst, lanes, (size_t)n * lanes, 1, 0, s);
}

// dlog[x] = log_3 x for x in [1, 65536] (3 generates GF(65537)*).
const std::vector<uint16_t>& dlog_table() {
  static const std::vector<uint16_t> t = [] {
    std::vector<uint16_t> v(65537, 0);
    uint32_t x = 1;
    for (uint32_t e = 0; e < 65536; ++e, x = x * 3u % 65537u) v[x] = (uint16_t)e;
    return v;
  }();
  return t;
}

// The table FNT_n(plane_b(l)), [n][16], l(d) = log(r_n^d - 1), l(0) = 0: built
// on first use for this n (host planes, one 16-lane transform, synchronised)
// and kept with the context.  `scr`: four-step scratch of the caller.
int conv_table(fntrs_ctx* c, int logn, uint32_t* scr, hipStream_t s) {
  if (c->conv_tab[logn]) return FNTRS_OK;
  const uint32_t n = 1u << logn;
  const auto& lg = dlog_table();
  uint64_t r = 1;
  for (uint32_t e = 0; e < (65536u >> logn); ++e) r = r * 3u % 65537u;   // r_n
  std::vector<uint32_t> planes((size_t)n * 16);
  uint64_t x = 1;
  for (uint32_t d = 0; d < n; ++d, x = x * r % 65537u) {
    const uint32_t l = d ? lg[(x + 65536u) % 65537u] : 0u;   // log(r_n^d - 1)
    for (int b = 0; b < 16; ++b) planes[(size_t)d * 16 + b] = (l >> b) & 1u;
  }
  const size_t bytes = planes.size() * 4;
  uint32_t *T = nullptr, *tmp = nullptr;
  if (hipMalloc((void**)&T, bytes) != hipSuccess) return fail(c, FNTRS_E_NOMEM, "hipMalloc(%zu) for the log table", bytes);
  if (hipMalloc((void**)&tmp, bytes) != hipSuccess) {
    (void)hipFree(T);
    return fail(c, FNTRS_E_NOMEM, "hipMalloc(%zu) for the log planes", bytes);
  }
  int rc = FNTRS_OK;
  if (hipMemcpyAsync(tmp, planes.data(), bytes, hipMemcpyHostToDevice, s) != hipSuccess)
    rc = fail(c, FNTRS_E_DEVICE, "log planes upload failed");
  if (!rc) rc = conv_fnt(c, n, 16, tmp, T, scr, s);
  if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "log table transform failed");
  (void)hipFree(tmp);
  if (rc) {
    (void)hipFree(T);
    return rc;
  }
  c->conv_tab[logn] = T;
  c->used += bytes;
  return FNTRS_OK;
}

// Steps 1-3 of one pattern from logarithms (the identities at k_conv_mark);
// d.zin holds its positions on the device and bstart the first rank of each
// 256 positions (n/256 + 1 words), S = e sum z mod 65536.  A's values at the
// n-th roots stay in L->Avals; its coefficients wait for locator_coeffs.
int conv_locator(fntrs_ctx* c, fntrs_locator_t* L, const LocDesc& d, const uint32_t* bstart, uint32_t S,
                 hipStream_t s) {
  const uint32_t n = d.n;
  const size_t wn = n;   // n >= 2^12: every part stays 256-byte aligned
  const size_t fsw = n >= (1u << kFourStepMinLog) ? kFnOneScratchWords : 0;
  Scratch sc;
  if (int rc = scratch_acquire(c, (2 * wn + 32 * wn + fsw) * 4, s, sc)) return rc;
  uint32_t* ind = reinterpret_cast<uint32_t*>(sc.p);
  uint32_t* F = ind + wn;
  uint32_t* P = F + wn;
  uint32_t* Q = P + 16 * wn;
  uint32_t* fs = Q + 16 * wn;
  int rc = conv_table(c, d.logn, fs, s);
  const uint32_t blocks = n / 256;
  if (!rc) {
    hipLaunchKernelGGL(k_conv_mark, dim3(blocks), dim3(256), 0, s, d.zin, bstart, ind, d.pos, d.ridx);
    rc = conv_fnt(c, n, 1, ind, F, fs, s);
  }
  if (!rc) {
    hipLaunchKernelGGL(k_conv_mul, dim3(4 * blocks), dim3(256), 0, s, (const uint32_t*)F,
                       (const uint32_t*)c->conv_tab[d.logn], P, n);
    rc = conv_fnt(c, n, 16, P, Q, fs, s);
  }
  if (!rc) {
    ConvFinishArgs a{Q, ind, d.ridx, c->tw, d.w, d.wfull, d.ahat, d.ahat_br, d.ahat_s, L->Avals, S, d.kr, d.logn,
                     d.logm};
    hipLaunchKernelGGL(k_conv_finish, dim3(blocks), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "logarithmic locator kernels failed");
  }
  scratch_release(c, sc, s);
  if (!rc) L->coeffs_pending = true;
  return rc;
}

}  // namespace

int locator_coeffs(fntrs_ctx* c, const fntrs_locator_t* L, hipStream_t s) {
  if (!L->coeffs_pending) return FNTRS_OK;
  const uint32_t n = L->n;
  const size_t fsw = n >= (1u << kFourStepMinLog) ? kFnOneScratchWords : 0;
  Scratch sc;
  if (int rc = scratch_acquire(c, ((size_t)n + fsw) * 4, s, sc)) return rc;
  uint32_t* G = reinterpret_cast<uint32_t*>(sc.p);
  int rc = FNTRS_OK;
  if (hipStreamWaitEvent(s, L->ready, 0) != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "stream wait failed");
  if (!rc) rc = conv_fnt(c, n, 1, L->Avals, G, G + n, s);   // A = FNT_n of its values at negated indices / n
  if (!rc) {
    hipLaunchKernelGGL(k_conv_coef, dim3((L->k + 256) / 256), dim3(256), 0, s, (const uint32_t*)G, L->A, L->k, L->logn);
    if (hipGetLastError() != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "locator coefficients kernel failed");
  }
  if (!rc && hipEventRecord(L->ready, s) != hipSuccess) rc = fail(c, FNTRS_E_DEVICE, "event record failed");
  scratch_release(c, sc, s);
  if (!rc) L->coeffs_pending = false;
  return rc;
}


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
  if (L->slab) c->used -= L->bytes;
  for (DirectMat** m : {&L->direct_w, &L->direct_sys}) {
    if (*m) c->used -= direct_mat_bytes(*m);
    direct_mat_free(*m);
    *m = nullptr;
  }
  delete L;   // the slab goes with its last locator
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

namespace {

size_t round_words(size_t w) { return (w + 63) / 64 * 64; }   // 256-byte aligned views

// Words of device state of a locator: pos[k] wfull[n] ridx[n] ahat_br[M]
// ahat_s[M] A[k+1] w[k] ahat[M] (M = 0 when nothing is erased).
size_t state_words(const fntrs_locator_t* L) {
  const size_t n = L->n, k = L->k, M = (k < n) ? (size_t)1 << L->logm : 0;
  return round_words(k) + 2 * round_words(n) + 3 * round_words(M) + round_words(k + 1) + round_words(k);
}

struct Range {
  uint32_t first = 0, count = 0;
};

}  // namespace

// Builds the device state of the locators `Ls` (steps 1-3 of Sec. II-B and
// the tables of steps 4 and 6) with one launch per stage for all of them:
// patterns sorted by k (nothing-erased patterns last), so that every stage
// covers a contiguous range of the descriptor table.
static int build_locators(fntrs_ctx* c, std::vector<fntrs_locator_t*>& Ls, hipStream_t s) {
  std::stable_sort(Ls.begin(), Ls.end(), [](const fntrs_locator_t* a, const fntrs_locator_t* b) {
    const bool ia = a->k == a->n, ib = b->k == b->n;
    return ia != ib ? ib : a->k < b->k;
  });
  const uint32_t P = (uint32_t)Ls.size();
  uint32_t Pn = 0;   // patterns with erasures
  while (Pn < P && Ls[Pn]->k < Ls[Pn]->n) ++Pn;
  // one large pattern alone: logarithms instead of the product tree (its
  // state keeps A at the n-th roots for the coefficients, taken on first use)
  const bool conv = P == 1 && Pn == 1 && Ls[0]->n >= (1u << kConvMinLog);
  // persistent state: one slab for the batch
  size_t words = 0;
  for (auto* L : Ls) {
    const size_t sw = state_words(L) + (conv ? round_words(L->n) : 0);
    L->bytes = sw * 4;
    words += sw;
  }
  if (!make_room(c, words * 4))
    return fail(c, FNTRS_E_NOMEM, "locator state of %zu bytes exceeds the context cap (%zu used of %zu)", words * 4,
                c->used, c->cap);
  auto slab = std::make_shared<LocSlab>();
  if (hipMalloc((void**)&slab->mem, words * 4) != hipSuccess) {
    slab->mem = nullptr;
    return fail(c, FNTRS_E_NOMEM, "hipMalloc(%zu) for locator state failed", words * 4);
  }
  HIP_TRY(c, hipEventCreateWithFlags(&slab->ready, hipEventDisableTiming));
  // host image: descriptors, positions, stage start tables
  std::vector<LocDesc> desc(P);
  std::vector<uint32_t> zall;
  size_t scratch = 0;
  uint32_t* p = slab->mem;
  std::vector<size_t> zoff(P), soff(P);
  for (uint32_t i = 0; i < P; ++i) {
    fntrs_locator_t* L = Ls[i];
    const size_t n = L->n, k = L->k, M = (k < n) ? (size_t)1 << L->logm : 0;
    L->pos = p; p += round_words(k);
    L->wfull = p; p += round_words(n);
    L->ridx = p; p += round_words(n);
    L->ahat_br = p; p += round_words(M);
    L->ahat_s = p; p += round_words(M);
    L->A = p; p += round_words(k + 1);
    L->w = p; p += round_words(k);
    L->ahat = p; p += round_words(M);
    if (conv) {
      L->Avals = p;
      p += round_words(n);
    }
    L->slab = slab;
    L->ready = slab->ready;
    zoff[i] = zall.size();
    zall.insert(zall.end(), L->positions.begin(), L->positions.end());
    soff[i] = scratch;
    const size_t kt = pad_pow2(L->k);    // points of the product tree
    if (k < n) scratch += 3 * round_words(kt) + round_words(n);
    LocDesc& d = desc[i];
    d = LocDesc{};
    d.pos = L->pos; d.wfull = L->wfull; d.ridx = L->ridx; d.ahat_br = L->ahat_br; d.ahat_s = L->ahat_s;
    d.A = L->A; d.w = L->w; d.ahat = L->ahat;
    d.n = L->n; d.k = (uint32_t)kt; d.kr = L->k; d.G = std::min<uint32_t>((uint32_t)kt, 64);
    d.logn = L->logn; d.logk = L->logk; d.logm = L->logm;
  }
  // stage tables: (range of descriptors, start offsets relative to the range)
  std::vector<uint32_t> tab;
  struct Stage {
    Range r;
    size_t start_off;   // in words within tab
    uint32_t total;
  };
  auto add_stage = [&](Range r, auto per) {
    Stage st{r, tab.size(), 0};
    uint64_t acc = 0;
    for (uint32_t q = 0; q < r.count; ++q) {
      tab.push_back((uint32_t)acc);
      acc += per(Ls[r.first + q]);
    }
    tab.push_back((uint32_t)acc);
    st.total = (uint32_t)acc;
    return st;
  };
  const Stage prep = add_stage({0, P}, [](const fntrs_locator_t* L) { return (uint64_t)L->k + L->n; });
  const Stage leaves = add_stage({0, Pn}, [](const fntrs_locator_t* L) {
    return (uint64_t)pad_pow2(L->k) / std::min<uint32_t>(pad_pow2(L->k), 64);
  });
  std::vector<std::pair<int, Stage>> levels;   // (log2 d, stage)
  for (int logd = 6; logd <= 15; ++logd) {
    uint32_t first = 0;
    while (first < Pn && pad_pow2(Ls[first]->k) <= (1u << logd)) ++first;
    if (first == Pn) break;
    levels.emplace_back(logd, add_stage({first, Pn - first}, [logd](const fntrs_locator_t* L) {
                          return (uint64_t)pad_pow2(L->k) >> (logd + 1);
                        }));
  }
  const Stage deriv = add_stage({0, Pn}, [](const fntrs_locator_t* L) { return (uint64_t)pad_pow2(L->k); });
  std::vector<std::pair<int, Stage>> evals;   // (log2 of the tree size, stage)
  for (uint32_t first = 0; first < Pn;) {
    uint32_t last = first;
    while (last < Pn && Ls[last]->logk == Ls[first]->logk) ++last;
    evals.emplace_back(Ls[first]->logk, add_stage({first, last - first}, [](const fntrs_locator_t* L) {
                         return (uint64_t)(L->n >> L->logk) + ((1ull << L->logm) >> L->logk);
                       }));
    first = last;
  }
  const Stage weights = add_stage({0, Pn}, [](const fntrs_locator_t* L) { return (uint64_t)L->k; });
  const Stage ahat = add_stage({0, Pn}, [](const fntrs_locator_t* L) { return 1ull << L->logm; });
  if (conv) {
    // the logarithmic route: the mark kernel reads the first rank of every
    // 256 positions and the positions straight from pinned host memory, so
    // no copy to the device goes ahead of it
    const auto& z = Ls[0]->positions;
    const size_t nb = desc[0].n / 256 + 1;
    fntrs_ctx::StageSlot* slot = nullptr;
    if (int rc = stage_slot(c, (nb + z.size()) * 4, slot)) return rc;
    uint32_t* h = static_cast<uint32_t*>(slot->p);
    uint64_t sum = 0, q = 0;
    for (uint32_t b = 0; b < nb; ++b) {
      while (q < z.size() && z[q] < b * 256u) sum += z[q++];
      h[b] = (uint32_t)q;
    }
    std::copy(z.begin(), z.end(), h + nb);
    const uint32_t S = (uint32_t)(((sum % 65536u) * (65536u >> desc[0].logn)) & 0xFFFFu);
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, slot->p, 0) != hipSuccess)
      return fail(c, FNTRS_E_DEVICE, "no device address for the staged positions");
    LocDesc d = desc[0];
    d.zin = static_cast<const uint32_t*>(dp) + nb;
    int rc = conv_locator(c, Ls[0], d, static_cast<const uint32_t*>(dp), S, s);
    if (hipEventRecord(slot->ev, s) != hipSuccess && !rc) rc = fail(c, FNTRS_E_DEVICE, "event record failed");
    slot->pending = true;
    if (rc) return rc;
    if (hipEventRecord(slab->ready, s) != hipSuccess) return fail(c, FNTRS_E_DEVICE, "event record failed");
    c->used += Ls[0]->bytes;
    return FNTRS_OK;
  }
  // short codes: one workgroup per pattern runs every step (its LDS holds a
  // tree of n/2 points and an M-point transform, M <= n)
  const bool small = P > 0 && Pn == P && std::all_of(Ls.begin(), Ls.end(), [](const fntrs_locator_t* L) {
    return L->k < L->n && L->n <= kLocSmallN && 2 * pad_pow2(L->k) <= L->n && (1u << L->logm) <= L->n;
  });
  if (small && P == 1 && Ls[0]->k <= kLocSmallMaxK) {
    // one short pattern: descriptor and positions by value, nothing uploaded
    LocSmallOne one{};
    one.d = desc[0];
    std::copy(Ls[0]->positions.begin(), Ls[0]->positions.end(), one.z);
    hipLaunchKernelGGL(k_locb_small1, dim3(1), dim3(kLocSmallNT), 0, s, one, (const uint32_t*)c->tw);
    if (hipError_t le = hipGetLastError(); le != hipSuccess)
      return fail(c, FNTRS_E_DEVICE, "locator kernel: %s", hipGetErrorString(le));
    if (hipEventRecord(slab->ready, s) != hipSuccess) return fail(c, FNTRS_E_DEVICE, "event record failed");
    c->used += Ls[0]->bytes;
    return FNTRS_OK;
  }
  // one transient allocation: descriptors | positions | tables | scratch
  const size_t desc_bytes = (P * sizeof(LocDesc) + 255) / 256 * 256;
  const size_t z_words = round_words(zall.size()), tab_words = round_words(tab.size());
  const size_t tmp_bytes = desc_bytes + (z_words + tab_words + scratch) * 4;
  Scratch tsc;
  if (int rc = scratch_acquire(c, tmp_bytes, s, tsc)) return rc;
  uint8_t* tmp = tsc.p;
  uint32_t* dz = reinterpret_cast<uint32_t*>(tmp + desc_bytes);
  uint32_t* dtab = dz + z_words;
  uint32_t* dscr = dtab + tab_words;
  for (uint32_t i = 0; i < P; ++i) {
    LocDesc& d = desc[i];
    d.zin = dz + zoff[i];
    if (d.kr < d.n) {   // an erasure pattern: the scratch reserved under L->k < L->n
      uint32_t* q = dscr + soff[i];
      const size_t kw = round_words(d.k);
      d.t0 = q; d.t1 = q + kw; d.spec = q + 2 * kw; d.vals = q + 3 * kw;
      const int nlev = ilog2(d.k / d.G);
      d.poly = (nlev & 1) ? d.t1 : d.t0;
    }
  }
  std::vector<uint8_t> img(tmp_bytes - scratch * 4, 0);
  std::memcpy(img.data(), desc.data(), P * sizeof(LocDesc));
  std::memcpy(img.data() + desc_bytes, zall.data(), zall.size() * 4);
  std::memcpy(img.data() + desc_bytes + z_words * 4, tab.data(), tab.size() * 4);
  auto release_tmp = [&]() { scratch_release(c, tsc, s); };
  auto fail_free = [&](int rc) {
    release_tmp();
    return rc;
  };
  if (int rc = upload_async(c, tmp, img.data(), img.size(), s)) return fail_free(rc);
  const LocDesc* D = reinterpret_cast<const LocDesc*>(tmp);
  auto launch_err = [&]() { return hipGetLastError(); };
  auto st_ptr = [&](const Stage& st) { return dtab + st.start_off; };
  const uint32_t* tw = c->tw;
  if (small) {
    hipLaunchKernelGGL(k_locb_small, dim3(P), dim3(kLocSmallNT), 0, s, D, tw);
  } else {
    hipLaunchKernelGGL(k_locb_prep, dim3((prep.total + 255) / 256), dim3(256), 0, s, D, st_ptr(prep), P);
    if (Pn) {
      hipLaunchKernelGGL(k_locb_leaves, dim3(leaves.total), dim3(64), 0, s, D, st_ptr(leaves), Pn, tw);
      // one pattern with a tree of 2^14 points or more: the top level and
      // the evaluations on the four-step kernels
      const bool one_big = Pn == 1 && desc[0].k >= (1u << 14);
      Scratch fsc;   // the four-step passes' rows, reused by each transform in turn
      if (one_big)
        if (int rc = scratch_acquire(c, kFnOneScratchWords * 4, s, fsc)) return fail_free(rc);
      uint32_t* fscr = reinterpret_cast<uint32_t*>(fsc.p);
      auto fail_both = [&](int rc) {
        scratch_release(c, fsc, s);
        return fail_free(rc);
      };
      for (size_t j = 0; j < levels.size(); ++j) {
        const int logd = levels[j].first;
        const Stage& st = levels[j].second;
        const uint32_t d = 1u << logd;
        if (one_big && 2 * d == desc[0].k) {
          if (int rc = top_level_fourstep(c, desc[0], (int)j, d, fscr, s)) return fail_both(rc);
          continue;
        }
        if (!level_ct(logd + 1, st.total, D + st.r.first, st_ptr(st), st.r.count, (int)j, tw, c->twi, s)) {
          const size_t lds = 2ull * d * 4;
          (void)set_lds_attr((const void*)k_locb_level, lds);
          const int nt = (int)std::min<uint32_t>(1024, std::max<uint32_t>(64, d / 2));
          hipLaunchKernelGGL(k_locb_level, dim3(st.total), dim3(nt), lds, s, D + st.r.first, st_ptr(st), st.r.count,
                             logd, (int)j, tw);
        }
      }
      hipLaunchKernelGGL(k_locb_derivative, dim3((deriv.total + 255) / 256), dim3(256), 0, s, D, st_ptr(deriv), Pn);
      for (auto& ev : evals) {
        if (one_big) {   // A' at the n-th roots, A mod x^kr at the M-th roots
          const LocDesc& d0 = desc[0];
          if (int rc = fnt_one(c, d0.n, d0.k, d0.spec, d0.vals, fscr, s)) return fail_both(rc);
          if (int rc = fnt_one(c, 1u << d0.logm, d0.kr, d0.A, d0.ahat, fscr, s)) return fail_both(rc);
          continue;
        }
        if (eval_ct(ev.first, ev.second.total, D + ev.second.r.first, st_ptr(ev.second), ev.second.r.count, tw, c->twi,
                    s))
          continue;
        const uint32_t K = 1u << ev.first;
        const size_t lds = (size_t)K * 4;
        (void)set_lds_attr((const void*)k_locb_eval, lds);
        const int nt = (int)std::min<uint32_t>(1024, std::max<uint32_t>(64, K / 4));
        hipLaunchKernelGGL(k_locb_eval, dim3(ev.second.total), dim3(nt), lds, s, D + ev.second.r.first,
                           st_ptr(ev.second), ev.second.r.count, ev.first, tw);
      }
      hipLaunchKernelGGL(k_locb_weights, dim3((weights.total + 255) / 256), dim3(256), 0, s, D, st_ptr(weights), Pn,
                         tw);
      hipLaunchKernelGGL(k_locb_ahat, dim3((ahat.total + 255) / 256), dim3(256), 0, s, D, st_ptr(ahat), Pn);
      scratch_release(c, fsc, s);
    }
  }
  if (hipError_t le = launch_err(); le != hipSuccess)
    return fail_free(fail(c, FNTRS_E_DEVICE, "locator kernels: %s", hipGetErrorString(le)));
  if (hipEventRecord(slab->ready, s) != hipSuccess) return fail_free(fail(c, FNTRS_E_DEVICE, "event record failed"));
  release_tmp();
  for (auto* L : Ls) c->used += L->bytes;
  return FNTRS_OK;
}

hipError_t launch_copy(const uint32_t* src, size_t stride_src, uint32_t* dst, size_t stride_dst, uint32_t lanes,
                       uint32_t batch, hipStream_t s) {
  const uint64_t total = (uint64_t)lanes * batch;
  hipLaunchKernelGGL(k_copy_rows, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, src, (uint64_t)stride_src,
                     dst, (uint64_t)stride_dst, lanes, batch, (const uint32_t*)nullptr);
  return hipGetLastError();
}

int locators_acquire(fntrs_ctx* c, uint32_t count, const uint32_t* n_, const uint32_t* k_,
                     const uint32_t* const* positions_, const uint32_t* npos_, hipStream_t stream,
                     fntrs_locator_t** out) {
  if (!out) return fail(c, FNTRS_E_INVAL, "null out");
  if (count && (!n_ || !k_ || !positions_ || !npos_)) return fail(c, FNTRS_E_INVAL, "null argument array");
  for (uint32_t q = 0; q < count; ++q) out[q] = nullptr;
  auto give_back = [&](uint32_t upto) {
    for (uint32_t q = 0; q < upto; ++q)
      if (out[q]) { out[q]->refs--; out[q] = nullptr; }
  };
  std::vector<fntrs_locator_t*> fresh;   // not cached: built below
  for (uint32_t q = 0; q < count; ++q) {
    const uint32_t n = n_[q], k = k_[q], npos = npos_[q];
    const uint32_t* positions = positions_[q];
    int rc = FNTRS_OK;
    if (n < 1 || n > 65536) rc = fail(c, FNTRS_E_INVAL, "n=%u must lie in [1, 65536]", n);
    else if (k < 1 || k > n) rc = fail(c, FNTRS_E_INVAL, "k=%u must satisfy 1 <= k <= n=%u", k, n);
    else if (!positions) rc = fail(c, FNTRS_E_INVAL, "null positions");
    else if (npos < k) rc = fail(c, FNTRS_E_TOOFEW, "%u positions received, k=%u needed", npos, k);
    else if (k < pad_pow2(n) && 2 * pad_pow2(k) > pad_pow2(n))
      rc = fail(c, FNTRS_E_UNSUPPORTED,
                "k=%u above half the transform length %u (k not a power of two, or 32768 < k < n): "
                "the low product would be longer than the transform", k, pad_pow2(n));
    for (uint32_t i = 0; !rc && i < k; ++i) {
      if (positions[i] >= n) rc = fail(c, FNTRS_E_POSITIONS, "position %u at index %u is >= n=%u", positions[i], i, n);
      else if (i && positions[i] <= positions[i - 1])
        rc = fail(c, FNTRS_E_POSITIONS, "positions must be strictly ascending (index %u)", i);
    }
    if (rc) {
      if (count > 1) c->err = "pattern " + std::to_string(q) + ": " + c->err;
      give_back(q);
      for (auto* L : fresh) delete L;
      return rc;
    }
    const uint64_t key = hash_positions(n, k, positions);
    auto same = [&](const fntrs_locator_t* L) {
      return L->nrows == n && L->k == k && std::equal(L->positions.begin(), L->positions.end(), positions);
    };
    fntrs_locator_t* hit = nullptr;
    auto range = c->cache.equal_range(key);
    for (auto it = range.first; it != range.second && !hit; ++it)
      if (same(it->second)) hit = it->second;
    for (auto* L : fresh)
      if (!hit && L->key == key && same(L)) hit = L;
    if (!hit) {
      hit = new fntrs_locator_t();
      hit->n = pad_pow2(n); hit->nrows = n; hit->k = k; hit->logn = ilog2(n); hit->logk = ilog2(k);
      hit->logm = std::max(hit->logk + 1, hit->logn - 1);   // low-product length M >= 2k, M >= n/2
      hit->positions.assign(positions, positions + k);
      hit->key = key;
      fresh.push_back(hit);
    }
    hit->refs++;
    hit->last_use = ++c->tick;
    out[q] = hit;
  }
  if (!fresh.empty()) {
    int rc = FNTRS_OK;
    if (c->device == FNTRS_HOST_ONLY) rc = fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
    else {
      DeviceGuard g(c->device);
      rc = build_locators(c, fresh, stream);
    }
    if (rc) {
      for (uint32_t q = 0; q < count; ++q)
        if (out[q] && std::find(fresh.begin(), fresh.end(), out[q]) == fresh.end()) out[q]->refs--;
      for (uint32_t q = 0; q < count; ++q) out[q] = nullptr;
      for (auto* L : fresh) delete L;   // not yet counted in c->used
      return rc;
    }
    for (auto* L : fresh) c->cache.emplace(L->key, L);
  }
  return FNTRS_OK;
}

// Default kernel configuration per transform size, then the FNTRS_TILES
// override "e12=8x512,d13=4x1024,d13=4x512v2,..." (tile lanes x threads, optional
// lanes per thread).
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
      int L = 0, T = 0, NT = 512, V = 0;
      char kind = 0;
      if (sscanf(item.c_str(), "%c%d=%dx%dv%d", &kind, &L, &T, &NT, &V) >= 3 && L >= 1 && L <= 15) {
        if (kind == 'e') c->enc_cfg[L] = CtCfg{T, NT, V};
        if (kind == 'd') c->dec_cfg[L] = CtCfg{T, NT, V};
      }
      pos = end + 1;
    }
  }
}

}  // namespace fntrs

using namespace fntrs;

// Scratch of fntrs_encode_noalloc: the intermediate rows of the four-step
// encoder (transforms of 2^14 points or more), batch * N * ceil32(lanes)
// words.  A file-scope device array, so that the entry point allocates
// nothing; every GPU the library runs on holds its own copy until the
// process ends, and every call on that GPU shares it.
constexpr size_t kNoAllocScratchWords = size_t(32) << 20;   // 128 MiB
static __device__ __align__(256) uint32_t scratch[kNoAllocScratchWords];

// Device address of `scratch` on each device, looked up once per device
// with that device current (the host-side name is not a device address).
static std::mutex g_scratch_mu;
static std::map<int, uint32_t*> g_scratch_ptr;

static int noalloc_scratch_init(fntrs_ctx* c) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(c->device);
  if (it == g_scratch_ptr.end()) {
    uint32_t* p = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(c, FNTRS_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    it = g_scratch_ptr.emplace(c->device, p).first;
  }
  c->noalloc_scratch = it->second;
  return FNTRS_OK;
}

// Encoder on validated arguments, enqueued on s; rows_out > 0 writes only
// the rows i < rows_out of dst.
int fntrs::encode_run(fntrs_ctx* c, uint32_t n, uint32_t k, uint32_t lanes, const uint32_t* src, size_t ld_src,
               size_t stride_src, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch, uint32_t rows_out,
               hipStream_t s, uint32_t* fixed_scratch) {
  if (n == 1) {  // k = 1: e_0 = s_0
    HIP_TRY(c, launch_copy(src, stride_src, dst, stride_dst, lanes, batch, s));
    return FNTRS_OK;
  }
  EncodeArgs a{};
  a.rows_out = rows_out;
  a.src = src; a.ld_src = ld_src; a.stride_src = stride_src;
  a.dst = dst; a.ld_dst = ld_dst; a.stride_dst = stride_dst;
  a.tw = c->tw; a.twi = c->twi;
  a.n = n; a.k = k; a.lanes = lanes;
  a.logn = ilog2(n);
  a.logK = std::max(1, ilog2(k));        // transform size K: smallest power of two >= k, at least 2
  if (encode_fourstep(c, a.logK, a.logn)) {
    // K >= 2^14: one FNT_n of the zero-padded source as four-step passes over
    // 32-lane tiles, through a scratch buffer
    FourStepArgs f{};
    f.in = src; f.ld_in = ld_src; f.stride_in = stride_src;
    f.out = dst; f.ld_out = ld_dst; f.stride_out = stride_dst;
    f.tw = c->tw; f.twi = c->twi;
    f.n = n; f.k = k; f.M = n; f.lanes = lanes; f.logn = a.logn; f.logm = a.logn;
    f.tiles = (lanes + kFourStepTile - 1) / kFourStepTile;
    f.rows_out = rows_out;
    const uint64_t lds = (uint64_t)f.tiles * kFourStepTile;
    f.vec = aligned16(src, ld_src, stride_src) && aligned16(dst, ld_dst, stride_dst);
    if (fixed_scratch) {   // the caller's scratch (no allocation)
      HIP_TRY(c, fourstep_encode(f, batch, fixed_scratch, lds, s));
      return FNTRS_OK;
    }
    Scratch sc;
    if (int rc = scratch_acquire(c, (size_t)batch * n * lds * 4, s, sc)) return rc;
    const hipError_t e = fourstep_encode(f, batch, reinterpret_cast<uint32_t*>(sc.p), lds, s);
    scratch_release(c, sc, s);
    HIP_TRY(c, e);
    return FNTRS_OK;
  }
  a.cosets = n >> a.logK;
  const CtCfg cfg = call_cfg(c, c->enc_cfg[a.logK], a.logK, lanes, (uint64_t)a.cosets * batch);
  a.vec = aligned16(src, ld_src, stride_src) && aligned16(dst, ld_dst, stride_dst);
  a.tiles = (lanes + cfg.T - 1) / cfg.T;
  const uint64_t blocks = (uint64_t)a.tiles * a.cosets * batch;
  if (blocks > 0x7fffffffull) return fail(c, FNTRS_E_INVAL, "grid too large");
  HIP_TRY(c, launch_ct_encode(c, a.logK, cfg, a, blocks, s));
  return FNTRS_OK;
}


// Decoder on validated arguments, enqueued on s.
int fntrs::decode_run(fntrs_ctx* c, const fntrs_locator_t* L, uint32_t lanes, bool full, const uint32_t* recv,
               size_t ld_recv, size_t stride_recv, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
               hipStream_t s) {
  const uint32_t n = L->n, k = L->k;
  HIP_TRY(c, hipStreamWaitEvent(s, L->ready, 0));
  if (n == 1) {  // k = n = 1: s_0 = e_0
    HIP_TRY(c, launch_copy(recv, stride_recv, dst, stride_dst, lanes, batch, s));
    return FNTRS_OK;
  }
  if (L->logn >= kFourStepMinLog) {
    FourStepArgs f{};
    f.in = recv; f.ld_in = ld_recv; f.stride_in = stride_recv;
    f.out = dst; f.ld_out = ld_dst; f.stride_out = stride_dst;
    f.tw = c->tw; f.twi = c->twi; f.wfull = L->wfull; f.ridx = L->ridx; f.ahat = L->ahat_s;
    f.n = n; f.k = k; f.lanes = lanes; f.logn = L->logn;
    f.logm = (k == n) ? L->logn : L->logm;
    f.M = 1u << f.logm;
    f.full = full ? 1u : 0u;
    f.tiles = (lanes + kFourStepTile - 1) / kFourStepTile;
    const uint64_t lds = (uint64_t)f.tiles * kFourStepTile;
    f.vec = aligned16(recv, ld_recv, stride_recv) && aligned16(dst, ld_dst, stride_dst);
    Scratch sc;
    if (int rc = scratch_acquire(c, (size_t)batch * (n + f.M) * lds * 4, s, sc)) return rc;
    uint32_t* sa = reinterpret_cast<uint32_t*>(sc.p);
    const hipError_t e = fourstep_decode(f, batch, sa, sa + (size_t)batch * n * lds, lds, s);
    scratch_release(c, sc, s);
    HIP_TRY(c, e);
    return FNTRS_OK;
  }
  DecodeArgs a{};
  a.recv = recv; a.ld_recv = ld_recv; a.stride_recv = stride_recv;
  a.dst = dst; a.ld_dst = ld_dst; a.stride_dst = stride_dst;
  a.tw = c->tw; a.twi = c->twi; a.wfull = L->wfull; a.ridx = L->ridx; a.ahat_br = L->ahat_br;
  a.n = n; a.k = k; a.lanes = lanes; a.logn = L->logn; a.logk = L->logk;
  a.full = full ? 1u : 0u;
  a.row0 = full ? L->positions[0] : 0u;
  const int D = (k == n) ? -1 : L->logn - L->logm;
  const CtCfg cfg = call_cfg(c, c->dec_cfg[L->logn], L->logn, lanes, batch);
  a.vec = aligned16(recv, ld_recv, stride_recv) && aligned16(dst, ld_dst, stride_dst);
  a.tiles = (lanes + cfg.T - 1) / cfg.T;
  const uint64_t blocks = (uint64_t)a.tiles * batch;
  if (blocks > 0x7fffffffull) return fail(c, FNTRS_E_INVAL, "grid too large");
  // A large call reads the (weight, row) pairs of its first pass from one
  // table in that pass's order (k_dec_pairs) instead of two tables at
  // bit-reversed positions: a wave's reads then share cache lines.
  if ((uint64_t)lanes * batch >= kDecPairsMinLanes && n >= 2 && n == (1u << L->logn)) {
    Scratch sc;
    if (int rc = scratch_acquire(c, (size_t)n * 8, s, sc)) return rc;
    uint32_t* wrb = reinterpret_cast<uint32_t*>(sc.p);
    hipLaunchKernelGGL(k_dec_pairs, dim3(std::min<uint32_t>(1024, (n + 255) / 256)), dim3(256), 0, s, L->wfull, L->ridx,
                       wrb, n, (int)L->logn, a.full);
    hipError_t e = hipGetLastError();
    a.wrb = wrb;
    if (e == hipSuccess) e = launch_ct_decode(c, L->logn, cfg, D, a, blocks, s);
    scratch_release(c, sc, s);
    HIP_TRY(c, e);
    return FNTRS_OK;
  }
  HIP_TRY(c, launch_ct_decode(c, L->logn, cfg, D, a, blocks, s));
  return FNTRS_OK;
}


// Systematic code (Sec. II-C), encoder: the source, read as the symbols
// received at positions 0..k-1, is interpolated into k intermediate symbols
// (the decoder with the locator of that pattern, cached in the context),
// whose transform is the codeword; its first k rows are the source.
static int systematic_encode_run(fntrs_ctx* c, uint32_t n, uint32_t k, uint32_t lanes, const uint32_t* src,
                                 size_t ld_src, size_t stride_src, uint32_t* dst, size_t ld_dst, size_t stride_dst,
                                 uint32_t batch, hipStream_t s) {
  std::vector<uint32_t> first(k);
  for (uint32_t i = 0; i < k; ++i) first[i] = i;
  const uint32_t* fp = first.data();
  fntrs_locator_t* L = nullptr;
  if (int rc = locators_acquire(c, 1, &n, &k, &fp, &k, s, &L)) return rc;
  Scratch sc;   // intermediate symbols [batch][k][lanes]
  int rc = scratch_acquire(c, (size_t)batch * k * lanes * 4, s, sc);
  if (!rc) {
    uint32_t* mid = reinterpret_cast<uint32_t*>(sc.p);
    rc = decode_run(c, L, lanes, false, src, ld_src, stride_src, mid, lanes, (size_t)k * lanes, batch, s);
    if (!rc)
      rc = encode_run(c, L->n, k, lanes, mid, lanes, (size_t)k * lanes, dst, ld_dst, stride_dst, batch,
                      n < L->n ? n : 0, s);
    scratch_release(c, sc, s);
  }
  L->refs--;
  return rc;
}

// Systematic code (Sec. II-C), decoder: the intermediate symbols from the k
// received symbols, then their transform at the first k positions.
static int systematic_decode_run(fntrs_ctx* c, const fntrs_locator_t* L, uint32_t lanes, bool full,
                                 const uint32_t* recv, size_t ld_recv, size_t stride_recv, uint32_t* dst,
                                 size_t ld_dst, size_t stride_dst, uint32_t batch, hipStream_t s) {
  const uint32_t n = L->n, k = L->k;
  Scratch sc;   // intermediate symbols [batch][k][lanes]
  if (int rc = scratch_acquire(c, (size_t)batch * k * lanes * 4, s, sc)) return rc;
  uint32_t* mid = reinterpret_cast<uint32_t*>(sc.p);
  int rc = decode_run(c, L, lanes, full, recv, ld_recv, stride_recv, mid, lanes, (size_t)k * lanes, batch, s);
  if (!rc) rc = encode_run(c, n, k, lanes, mid, lanes, (size_t)k * lanes, dst, ld_dst, stride_dst, batch, k, s);
  scratch_release(c, sc, s);
  return rc;
}

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
  // Stream-ordered scratch (locator builds, batch tables, four-step passes)
  // is allocated and freed per call.  With the pool's default release
  // threshold of 0 every free hands the memory back to the driver (~15 us a
  // call); keep up to the workspace cap reserved in the device's pool.
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
    uint64_t keep = c->cap;
    uint64_t cur = 0;
    if (hipMemPoolGetAttribute(pool, hipMemPoolAttrReleaseThreshold, &cur) == hipSuccess && cur < keep)
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  // twiddle tables: tw[e] = 3^e and twi[e] = 3^-e = 3^(65536-e), e < 65536
  std::vector<uint32_t> h(2 * 65536);
  uint64_t x = 1;
  for (int e = 0; e < 65536; ++e) { h[e] = (uint32_t)x; x = x * 3 % 65537; }
  for (int e = 0; e < 65536; ++e) h[65536 + e] = h[(65536 - e) & 0xFFFF];
  // the stage tables (stage_tw_offset), then the four-step split twiddles
  // (split_tw_offset): w_N^(+-i t) by [i][t]
  h.resize(kStageTwBase + kStageTwWords + kSplitTwWords);
  for (int lg = 1; lg <= 16; ++lg)
    for (uint32_t j = 0; j <= (1u << (lg - 1)); ++j) h[kStageTwBase + stage_tw_offset(lg) + j] = h[j << (16 - lg)];
  for (int logN = kSplitTwMinLog; logN <= 16; ++logN) {
    const uint32_t N = 1u << logN, N2 = N >> 8, sh = 16 - logN;
    for (int b = 0; b < 2; ++b)
      for (int inv = 0; inv < 2; ++inv) {
        uint32_t* t = h.data() + split_tw_offset(logN, b != 0, inv != 0);
        const uint32_t rows = b ? 256 : N2, cols = b ? N2 : 256;
        for (uint32_t i = 0; i < rows; ++i)
          for (uint32_t j = 0; j < cols; ++j) t[i * cols + j] = h[(inv ? 65536 : 0) + (((i * j) & (N - 1)) << sh)];
      }
  }
  const size_t tw_bytes = h.size() * 4;
  if (hipMalloc((void**)&c->tw, tw_bytes) != hipSuccess) { delete c; return FNTRS_E_NOMEM; }
  c->twi = c->tw + 65536;
  c->used += tw_bytes;
  if (hipMemcpy(c->tw, h.data(), tw_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(c->tw);
    delete c;
    return FNTRS_E_DEVICE;
  }
  if (noalloc_scratch_init(c) != FNTRS_OK) {
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
  for (auto& kv : c->parity) direct_mat_free(kv.second);
  c->parity.clear();
  auto drop = [](fntrs_ctx::SideSet& ss) {
    for (int b = 0; b < fntrs_ctx::kSide; ++b) {
      if (ss.st[b]) (void)hipStreamDestroy(ss.st[b]);
      if (ss.join[b]) (void)hipEventDestroy(ss.join[b]);
    }
    if (ss.fork) (void)hipEventDestroy(ss.fork);
  };
  for (auto& kv : c->sides) drop(kv.second);
  drop(c->capture_side);
  stage_release(c);
  workspace_release(c);
  for (uint32_t* t : c->conv_tab)
    if (t) (void)hipFree(t);
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
  if (!(flags & (FNTRS_DIRECT | FNTRS_TRANSFORM | FNTRS_SYSTEMATIC)) && direct_fits(pad_pow2(n), k) &&
      c->use_direct[FNTRS_OP_ENCODE][std::max(1, ilog2(k))])
    flags |= FNTRS_DIRECT;   // the autotuner found the direct method faster for this class
  if (flags & FNTRS_DIRECT) {   // the quadratic methods of Sec. III
    const uint32_t N = pad_pow2(n);
    if (!direct_fits(N, k))
      return fail(c, FNTRS_E_UNSUPPORTED, "direct encoding covers k <= %u and n <= %u (k=%u n=%u)", kDirectMaxK,
                  kDirectMaxN, k, n);
    if (flags & FNTRS_SYSTEMATIC)
      return direct_systematic_encode(c, N, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, s);
    return direct_encode(c, N, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, s);
  }
  if (flags & FNTRS_SYSTEMATIC)
    return systematic_encode_run(c, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, s);
  const uint32_t N = pad_pow2(n);   // a shorter code: the rows n..N-1 are not written
  return encode_run(c, N, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, n < N ? n : 0, s);
}

int fntrs_encode_noalloc(fntrs_ctx* c, uint32_t n, uint32_t k, uint32_t lanes, const uint32_t* src, size_t ld_src,
                         size_t stride_src, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
                         uint32_t flags, void* stream) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (flags) return fail(c, FNTRS_E_INVAL, "fntrs_encode_noalloc takes no flags (got 0x%x)", flags);
  if (int rc = check_encode(c, n, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, 0)) return rc;
  const uint32_t N = pad_pow2(n);
  const int logK = std::max(1, ilog2(k));
  const bool fourstep = N > 1 && encode_fourstep(c, logK, ilog2(N));
  const size_t words =
      fourstep ? (size_t)batch * N * ((lanes + kFourStepTile - 1) / kFourStepTile * kFourStepTile) : 0;
  if (words > kNoAllocScratchWords)
    return fail(c, FNTRS_E_NOMEM,
                "fntrs_encode_noalloc: the four-step scratch needs %zu words, above its fixed %zu "
                "(batch * N * lanes rounded up to 32)",
                words, kNoAllocScratchWords);
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
  if (!c->noalloc_scratch) return fail(c, FNTRS_E_DEVICE, "the no-allocation scratch has no device address");
  DeviceGuard g(c->device);
  return encode_run(c, N, k, lanes, src, ld_src, stride_src, dst, ld_dst, stride_dst, batch, n < N ? n : 0,
                    (hipStream_t)stream, c->noalloc_scratch);
}

int fntrs_locator(fntrs_ctx* c, uint32_t n, uint32_t k, const uint32_t* positions, uint32_t npos, void* stream,
                  fntrs_locator_t** out) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  if (!out) return fail(c, FNTRS_E_INVAL, "null out");
  return locators_acquire(c, 1, &n, &k, &positions, &npos, (hipStream_t)stream, out);
}

int fntrs_locator_batch(fntrs_ctx* c, uint32_t count, const uint32_t* n, const uint32_t* k,
                        const uint32_t* const* positions, const uint32_t* npos, void* stream,
                        fntrs_locator_t** out) {
  if (!c) return FNTRS_E_INVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  c->err.clear();
  return locators_acquire(c, count, n, k, positions, npos, (hipStream_t)stream, out);
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
  if (A)
    if (int rc = locator_coeffs(c, L, nullptr)) return rc;
  HIP_TRY(c, hipEventSynchronize(L->ready));
  if (A) HIP_TRY(c, hipMemcpy(A, L->A, (L->k + 1) * 4ull, hipMemcpyDeviceToHost));
  if (w) HIP_TRY(c, hipMemcpy(w, L->w, L->k * 4ull, hipMemcpyDeviceToHost));
  if (ahat && L->k != L->n && is_pow2(L->k)) {
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
  const uint32_t rrows = full ? L->nrows : L->k;
  if (c->device == FNTRS_HOST_ONLY) return fail(c, FNTRS_E_DEVICE, "host-only context: arguments valid, no device");
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  if (flags & FNTRS_FLAG_VALIDATE) {
    int rc = validate_range(c, recv, batch, stride_recv, rrows, ld_recv, lanes, s);
    if (rc) return rc;
  }
  if (!(flags & (FNTRS_DIRECT | FNTRS_TRANSFORM | FNTRS_SYSTEMATIC)) && L->k < L->n && direct_fits(L->n, L->k) &&
      c->use_direct[FNTRS_OP_DECODE][L->logn])
    flags |= FNTRS_DIRECT;   // the autotuner found the direct method faster for this class
  if (flags & FNTRS_DIRECT) {   // the quadratic methods of Sec. III
    if (L->k == L->n || !direct_fits(L->n, L->k))
      return fail(c, FNTRS_E_UNSUPPORTED, "direct decoding covers 1 <= k < n, k <= %u, n <= %u (k=%u n=%u)",
                  kDirectMaxK, kDirectMaxN, L->k, L->nrows);
    auto* Lm = const_cast<fntrs_locator_t*>(L);
    if (flags & FNTRS_SYSTEMATIC)
      return direct_systematic_decode(c, Lm, lanes, full, recv, ld_recv, stride_recv, dst, ld_dst, stride_dst, batch,
                                      s);
    return direct_decode(c, Lm, lanes, full, recv, ld_recv, stride_recv, dst, ld_dst, stride_dst, batch, s);
  }
  if (flags & FNTRS_SYSTEMATIC)
    return systematic_decode_run(c, L, lanes, full, recv, ld_recv, stride_recv, dst, ld_dst, stride_dst, batch, s);
  return decode_run(c, L, lanes, full, recv, ld_recv, stride_recv, dst, ld_dst, stride_dst, batch, s);
}

}  // extern "C"
