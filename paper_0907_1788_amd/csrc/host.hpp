// Host-side internals of libfntrs shared by its translation units: the
// context and locator objects, error reporting, argument checks.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "../../include/fntrs.h"
#include "ct_launch.hpp"
#include "fourstep_launch.hpp"

namespace fntrs {

constexpr size_t kDefaultCap = size_t(4) << 30;

inline bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }
inline int ilog2(uint64_t x) { int r = 0; while ((1ull << r) < x) ++r; return r; }
// Transform length of a code of length n: the smallest power of two >= n (a
// shorter code is the longer one with its last symbols never sent).
inline uint32_t pad_pow2(uint32_t n) { return n <= 1 ? 1u : 1u << ilog2(n); }

}  // namespace fntrs

// Device memory and completion event shared by the locators built together
// in one batch; freed when the last of them is.
struct LocSlab {
  uint32_t* mem = nullptr;
  hipEvent_t ready = nullptr;        // recorded after the build on its stream
  LocSlab() = default;
  LocSlab(const LocSlab&) = delete;
  LocSlab& operator=(const LocSlab&) = delete;
  ~LocSlab() {
    if (ready) (void)hipEventDestroy(ready);
    if (mem) (void)hipFree(mem);   // waits for work still using it
  }
};

namespace fntrs {
struct DirectMat;
void direct_mat_free(DirectMat* m);
size_t direct_mat_bytes(const DirectMat* m);
}  // namespace fntrs

struct fntrs_locator_s {
  uint32_t n = 0, k = 0;             // n: transform length, the power of two >= the code length
  uint32_t nrows = 0;                // the code length (rows of a full received buffer)
  int logn = 0, logk = 0;
  int logm = 0;                      // low-product length M = 2^logm >= 2k (k < n)
  std::vector<uint32_t> positions;   // the k positions used
  uint64_t key = 0;
  std::shared_ptr<LocSlab> slab;     // holds the views below
  size_t bytes = 0;                  // this locator's share of the slab
  uint32_t *pos = nullptr, *wfull = nullptr, *ridx = nullptr, *ahat_br = nullptr, *ahat_s = nullptr;
  uint32_t *A = nullptr, *w = nullptr, *ahat = nullptr;
  // logarithmic route: A at the n-th roots, and whether the coefficients A
  // still have to be taken from them (on first use: export, direct decoding)
  uint32_t* Avals = nullptr;
  mutable bool coeffs_pending = false;
  hipEvent_t ready = nullptr;        // the slab's event
  // direct (quadratic) decoders: the inverse of the received rows of the
  // generator, and the systematic decoder's matrix and row tables
  fntrs::DirectMat* direct_w = nullptr;
  fntrs::DirectMat* direct_sys = nullptr;
  uint32_t direct_e = 0, direct_g = 0;   // missing / received source positions
  int refs = 0;
  uint64_t last_use = 0;
};

struct fntrs_ctx {
  int device = 0;
  int num_cu = 256;
  size_t cap = fntrs::kDefaultCap, used = 0;
  uint32_t* tw = nullptr;            // tw[e] = 3^e mod p, e < 65536
  uint32_t* twi = nullptr;           // twi[e] = 3^-e mod p (tw + 65536; the four-step split
                                     // twiddles follow, see split_tw_offset)
  uint32_t* noalloc_scratch = nullptr;   // device address of the no-allocation encoder's scratch
  uint32_t* conv_tab[17] = {};       // per log2 n: FNT_n of the 16 bit planes of log(r_n^d - 1), [n][16]
  size_t lds_max = 65536;
  fntrs::CtCfg enc_cfg[16] = {};     // kernel configuration per log2 transform size
  fntrs::CtCfg dec_cfg[16] = {};
  bool use_direct[2][17] = {};       // autotuner: the class's single calls use the direct methods
  bool enc_fourstep13 = false;       // autotuner: encode K = 2^13 into n >= 2^14 as one four-step FNT_n
  std::mutex mu;
  std::string err;
  std::unordered_multimap<uint64_t, fntrs_locator_t*> cache;
  uint64_t tick = 0;
  // batched path: per caller stream, side streams (default priority) that
  // run a batch's size classes concurrently; one more set for captures
  static constexpr int kSide = 3;
  struct SideSet {
    hipStream_t st[kSide] = {};
    hipEvent_t fork = nullptr, join[kSide] = {};
  };
  std::unordered_map<hipStream_t, SideSet> sides;
  SideSet capture_side;
  // occupancy of each table kernel
  std::map<std::tuple<int, int, int, int, int>, int> occ;
  // pinned host staging for table uploads: a copy from pageable memory is
  // synchronous and would keep the host from running ahead of the device.
  // A slot is reused once the event recorded after its copy has fired.
  struct StageSlot {
    void* p = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
  };
  std::vector<StageSlot> stage;
  // device buffers for small per-call tables (locator builds, batch job
  // tables): allocating and freeing stream-ordered memory costs ~15 us of
  // host time a call.  A slot is reused once the event recorded after its
  // last use has fired.
  struct DevSlot {
    uint8_t* p = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool pending = false, busy = false;   // busy: held by a call (calls nest)
  };
  std::deque<DevSlot> dev_slots;
  // reusable device blocks for larger transient buffers (four-step scratch,
  // big batch tables, locator builds), held up to the workspace cap: a
  // serving loop then stops allocating once it has seen its largest batch
  // (new device memory can make the allocating call wait for the GPU).  A
  // block is busy while a call holds it and pending until the event recorded
  // after its last use has fired; a pending block is reused in stream order.
  struct WsBlock {
    uint8_t* p = nullptr;
    size_t bytes = 0;
    hipEvent_t ev = nullptr;
    bool pending = false, busy = false;
  };
  std::deque<WsBlock> ws;   // stable addresses: calls nest (systematic, chirp)
  size_t ws_held = 0;
  // direct systematic encoder: parity matrix per (N, k)
  std::map<std::pair<uint32_t, uint32_t>, fntrs::DirectMat*> parity;
};

namespace fntrs {

int fail(fntrs_ctx* c, int code, const char* fmt, ...) __attribute__((format(printf, 3, 4)));

#define HIP_TRY(ctx, expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(ctx, FNTRS_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

inline bool aligned16(const void* p, size_t ld, size_t stride) {
  return ((uintptr_t)p % 16 == 0) && (ld % 4 == 0) && (stride % 4 == 0);
}

inline bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes) {
  auto pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + bbytes && pb < pa + abytes;
}

inline size_t span_elems(uint32_t batch, size_t stride, uint32_t rows, size_t ld, uint32_t lanes) {
  return (size_t)(batch - 1) * stride + (size_t)(rows - 1) * ld + lanes;
}

struct CtTables {
  const CtEncLaunch* enc;
  const CtDecLaunch* dec;
  const CtEncTabLaunch* enc_tab;
  const CtDecTabLaunch* dec_tab;
  const CtEncCosLaunch* enc_cos;
  const CtDecPipeLaunch* dec_pipe;
  const CtTabOccupancy* occ;
  const CtEncCosTabLaunch* enc_cos_tab;
};
const CtTables& ct_tables();

// Enqueues a host-to-device copy of `bytes` bytes of `src` on `s` through a
// pinned staging slot (the host returns at once; the slot stays reserved
// until the copy has run).
int upload_async(fntrs_ctx* c, void* dst, const void* src, size_t bytes, hipStream_t s);
// Frees the staging slots (the device must be idle).
void stage_release(fntrs_ctx* c);

// Largest per-call table served from the device slots; larger buffers are
// allocated stream-ordered.
constexpr size_t kDevSlotMax = size_t(64) << 20;
// A device buffer of at least `bytes` (<= kDevSlotMax) idle on every stream;
// dev_slot_done must follow its last use on stream s.
int dev_slot_acquire(fntrs_ctx* c, size_t bytes, fntrs_ctx::DevSlot*& out);
int dev_slot_done(fntrs_ctx* c, fntrs_ctx::DevSlot* slot, hipStream_t s);

// A transient device buffer of a call: a device slot (small tables), a
// workspace block, or a stream-ordered allocation when no block fits under
// the cap.  scratch_release must follow its last use on stream s.
struct Scratch {
  uint8_t* p = nullptr;
  int kind = 0;            // 0 none, 1 device slot, 2 workspace block, 3 stream-ordered
  void* ref = nullptr;
};
int scratch_acquire(fntrs_ctx* c, size_t bytes, hipStream_t s, Scratch& out);
void scratch_release(fntrs_ctx* c, Scratch& sc, hipStream_t s);
// Frees the workspace blocks (the device must be idle).
void workspace_release(fntrs_ctx* c);

// The configuration of one single call of size 2^L (see ct_small).
CtCfg call_cfg(const fntrs_ctx* c, CtCfg cfg, int L, uint32_t lanes, uint64_t per);

// Resident workgroups per CU of a persistent kernel (cached per context);
// op 0/1 = encode/decode table kernel, 2 = pipelined decode kernel;
// 0 = not available.
int kernel_occupancy(fntrs_ctx* c, int op, int L, int D, CtCfg cfg);

// One encode / decode over `items` work items of the single job `a` with the
// compile-time kernels of size 2^L: the pipelined persistent kernel when the
// configuration has one, else one workgroup per work item.
hipError_t launch_ct_encode(fntrs_ctx* c, int L, CtCfg cfg, const EncodeArgs& a, uint64_t items, hipStream_t s);
hipError_t launch_ct_decode(fntrs_ctx* c, int L, CtCfg cfg, int D, const DecodeArgs& a, uint64_t items,
                            hipStream_t s);

// Argument checks of one encode / decode call (the rules of fntrs_encode and
// fntrs_decode); FNTRS_OK or an error code with the message set.
int check_encode(fntrs_ctx* c, uint32_t n, uint32_t k, uint32_t lanes, const uint32_t* src, size_t ld_src,
                 size_t stride_src, const uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
                 uint32_t flags);
int check_decode(fntrs_ctx* c, const fntrs_locator_t* L, uint32_t lanes, uint32_t flags, const uint32_t* recv,
                 size_t ld_recv, size_t stride_recv, const uint32_t* dst, size_t ld_dst, size_t stride_dst,
                 uint32_t batch);
// Reads a strided device region back and checks every residue <= 65536.
int validate_range(fntrs_ctx* c, const uint32_t* p, uint32_t batch, size_t stride, uint32_t rows, size_t ld,
                   uint32_t lanes, hipStream_t s);
// The transform encoder / decoder of one call on validated arguments (N a
// power of two; rows_out > 0 writes only rows < rows_out), enqueued on s.
// fixed_scratch: the four-step scratch to use instead of allocating one.
int encode_run(fntrs_ctx* c, uint32_t N, uint32_t k, uint32_t lanes, const uint32_t* src, size_t ld_src,
               size_t stride_src, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch, uint32_t rows_out,
               hipStream_t s, uint32_t* fixed_scratch = nullptr);
int decode_run(fntrs_ctx* c, const fntrs_locator_t* L, uint32_t lanes, bool full, const uint32_t* recv,
               size_t ld_recv, size_t stride_recv, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
               hipStream_t s);
// Whether an encode of transform size 2^logK into a code of transform length
// 2^logN runs as one four-step FNT_n: always from 2^14 points, and at 2^13
// when the autotuner found that faster (the four-step kernels need N >= 2^14).
inline bool encode_fourstep(const fntrs_ctx* c, int logK, int logN) {
  return logK >= kFourStepMinLog || (logK == kFourStepMinLog - 1 && logN >= kFourStepMinLog && c->enc_fourstep13);
}
// Direct (quadratic) methods of Sec. III (direct.hip), for codes with
// k <= kDirectMaxK and transform length N <= kDirectMaxN.
constexpr uint32_t kDirectMaxK = 1024, kDirectMaxN = 16384;
bool direct_fits(uint32_t N, uint32_t k);
// The coefficients of A for a locator of the logarithmic route, computed on
// `s` after the locator's build the first time they are needed; the
// locator's ready event then covers them.
int locator_coeffs(fntrs_ctx* c, const fntrs_locator_t* L, hipStream_t s);
int direct_encode(fntrs_ctx* c, uint32_t N, uint32_t rows, uint32_t k, uint32_t lanes, const uint32_t* src,
                  size_t ld_src, size_t stride_src, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch,
                  hipStream_t s);
int direct_decode(fntrs_ctx* c, fntrs_locator_t* L, uint32_t lanes, bool full, const uint32_t* recv, size_t ld_recv,
                  size_t stride_recv, uint32_t* dst, size_t ld_dst, size_t stride_dst, uint32_t batch, hipStream_t s);
int direct_systematic_encode(fntrs_ctx* c, uint32_t N, uint32_t rows, uint32_t k, uint32_t lanes,
                             const uint32_t* src, size_t ld_src, size_t stride_src, uint32_t* dst, size_t ld_dst,
                             size_t stride_dst, uint32_t batch, hipStream_t s);
int direct_systematic_decode(fntrs_ctx* c, fntrs_locator_t* L, uint32_t lanes, bool full, const uint32_t* recv,
                             size_t ld_recv, size_t stride_recv, uint32_t* dst, size_t ld_dst, size_t stride_dst,
                             uint32_t batch, hipStream_t s);
// Evicts unreferenced cached locators until `need` more bytes fit the cap.
bool make_room(fntrs_ctx* c, size_t need);
// Finds the cached locators of `count` patterns or builds the missing ones
// together (fntrs_locator_batch without the lock); all or nothing.
int locators_acquire(fntrs_ctx* c, uint32_t count, const uint32_t* n, const uint32_t* k,
                     const uint32_t* const* positions, const uint32_t* npos, hipStream_t stream,
                     fntrs_locator_t** out);
hipError_t launch_copy(const uint32_t* src, size_t stride_src, uint32_t* dst, size_t stride_dst, uint32_t lanes,
                       uint32_t batch, hipStream_t s);

}  // namespace fntrs
