// A stand-in for the HIP runtime that runs no GPU code: it checks the
// stream ordering and memory lifetimes of everything libfntrs enqueues.
//
// Built as a shared library with the soname of the HIP runtime, it is loaded
// in place of the real one by a process that drives libfntrs through its C
// ABI.  Streams are FIFO queues of operations; events and stream waits give
// each operation a vector clock (how many operations of every stream must
// have completed before it may start).  A simulated device executes the
// runnable operations lazily and in a seeded random order, so that the host
// runs ahead of the device the way it does on a GPU.  When an operation
// executes, every range of device or pinned memory it touches is checked:
//   - the range lies inside an allocation that is live at that moment (the
//     GPU's illegal-address fault, or a use after free);
//   - a stream-ordered allocation was made before it in stream order;
//   - every conflicting earlier access (one of the two a write) is ordered
//     before it by the streams and events, i.e. no data race;
//   - a host-to-device copy from pinned memory finds the bytes the host
//     gave it at enqueue time (the host has not reused the buffer early).
// Kernels are modelled by the memory their arguments say they touch: the
// argument structs are decoded from the launch, and device-side job and
// descriptor tables are read from the simulated memory when the kernel
// executes, as the GPU would read them.
//
// Control (C ABI): fakehip_seed, fakehip_set_lag, fakehip_drain,
// fakehip_errors, fakehip_error_text, fakehip_stats.
#include <hip/hip_runtime_api.h>
#include <sys/mman.h>

#include <cxxabi.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "kernel_args.hpp"

struct ihipStream_t {
  int id;
};
struct ihipEvent_t {
  int id;
};

namespace {

using fntrs::DecodeArgs;
using fntrs::EncodeArgs;
using fntrs::FourStepArgs;
using fntrs::GemmArgs;
using fntrs::JobTable;
using fntrs::LocDesc;

using Clock = std::vector<int64_t>;

int64_t at(const Clock& c, size_t i) { return i < c.size() ? c[i] : 0; }
void join(Clock& a, const Clock& b) {
  if (a.size() < b.size()) a.resize(b.size(), 0);
  for (size_t i = 0; i < b.size(); ++i) a[i] = std::max(a[i], b[i]);
}

struct Range {
  uintptr_t lo, hi;
  bool write;
};

struct Op {
  int stream = 0;
  int64_t seq = 0;   // 1-based position in its stream
  Clock clk;         // operations that must complete first
  std::string what;
  std::function<void(Op&)> run;
};

struct Stream {
  std::deque<std::unique_ptr<Op>> q;
  int64_t enq = 0, exec = 0;
  Clock clk;         // everything enqueued so far, and what it waits for
  bool destroyed = false;
};

struct Event {
  Clock clk;
  bool recorded = false;
};

struct Record {   // an executed access
  uintptr_t lo, hi;
  bool write;
  int stream;
  int64_t seq;
  std::string what;
};

struct Alloc {
  uintptr_t lo = 0, hi = 0;
  int kind = 0;                 // 0 device, 1 device stream-ordered, 2 pinned host, 3 device symbol
  bool freed = false;
  int alloc_stream = -1;        // stream-ordered: the allocating operation
  int64_t alloc_seq = 0;
  bool alloc_done = true;
  std::vector<Record> rec;
};

struct State {
  std::mutex mu;
  std::deque<Stream> streams;              // deque: elements never move
  std::vector<Event> events;
  Clock host;                             // operations the host has seen complete
  std::map<uintptr_t, Alloc> allocs;      // by lo
  std::map<const void*, std::string> kernels;
  std::map<const void*, std::pair<uintptr_t, size_t>> symbols;
  std::vector<std::string> errors;
  std::mt19937_64 rng{1};
  double lag = 0.7;                       // probability that a call leaves the device idle
  uintptr_t dev_next = 0, dev_end = 0;
  struct Cfg {
    dim3 g, b;
    size_t shm;
    hipStream_t s;
  };
  std::vector<Cfg> cfg;
  uint64_t ops_run = 0, kernels_run = 0, checks = 0;
  uint64_t n_malloc = 0, n_malloc_async = 0, n_wait_event = 0;   // call counts
  State() {
    streams.resize(1);   // the null stream
    const size_t span = size_t(1) << 42;   // 4 TiB of address space, touched pages only
    void* p = mmap(nullptr, span, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (p == MAP_FAILED) {
      fprintf(stderr, "fake_hip: cannot reserve the simulated device memory\n");
      abort();
    }
    dev_next = (uintptr_t)p;
    dev_end = dev_next + span;
  }
};

State& S() {
  static State s;
  return s;
}

void error(const std::string& m) {
  State& st = S();
  if (st.errors.size() < 200) st.errors.push_back(m);
}

int sid(hipStream_t s) { return s ? s->id : 0; }

Alloc* find_alloc(uintptr_t p) {
  State& st = S();
  auto it = st.allocs.upper_bound(p);
  if (it == st.allocs.begin()) return nullptr;
  --it;
  return (p >= it->second.lo && p < it->second.hi) ? &it->second : nullptr;
}

uintptr_t dev_alloc(size_t bytes, int kind) {
  State& st = S();
  const size_t sz = (std::max<size_t>(bytes, 1) + 4095) / 4096 * 4096;
  if (st.dev_next + sz + 4096 > st.dev_end) return 0;
  const uintptr_t p = st.dev_next;
  st.dev_next += sz + 4096;   // a guard page between allocations
  Alloc a;
  a.lo = p;
  a.hi = p + bytes;
  a.kind = kind;
  st.allocs[p] = a;
  return p;
}

bool hb(const Op& x, int stream, int64_t seq) { return stream == x.stream ? seq < x.seq : at(x.clk, stream) >= seq; }

std::string hexs(uintptr_t p) {
  char b[32];
  snprintf(b, sizeof b, "0x%zx", (size_t)p);
  return b;
}

// Checks one range of an executing operation and records the access.
void touch(Op& x, uintptr_t lo, size_t bytes, bool write, const char* what) {
  State& st = S();
  ++st.checks;
  if (bytes == 0) return;
  const uintptr_t hi = lo + bytes;
  Alloc* a = find_alloc(lo);
  const std::string where = x.what + " / " + what;
  if (!a || hi > a->hi) {
    error("out of bounds: " + where + " touches [" + hexs(lo) + ", " + hexs(hi) + ") outside any allocation" +
          (a ? " (runs past one of " + std::to_string(a->hi - a->lo) + " bytes by " + std::to_string(hi - a->hi) + ")"
             : ""));
    return;
  }
  if (a->freed) {
    error("use after free: " + where + " touches freed memory at " + hexs(lo));
    return;
  }
  if (a->kind == 1 && !(a->alloc_stream == x.stream ? a->alloc_seq < x.seq : at(x.clk, a->alloc_stream) >= a->alloc_seq))
    error("stream-ordered allocation used before its allocation in stream order: " + where);
  for (const Record& r : a->rec) {
    if (r.hi <= lo || r.lo >= hi) continue;
    if (!(r.write || write)) continue;
    if (r.stream == x.stream && r.seq == x.seq) continue;   // this operation's own earlier access
    if (!hb(x, r.stream, r.seq))
      error(std::string("race: ") + where + (write ? " writes " : " reads ") + "[" + hexs(lo) + ", " + hexs(hi) +
            ") against " + (r.write ? "a write" : "a read") + " by " + r.what + " that is not ordered before it");
  }
  // keep the list short: drop what this access supersedes
  auto& rec = a->rec;
  rec.erase(std::remove_if(rec.begin(), rec.end(),
                           [&](const Record& r) {
                             if (r.lo < lo || r.hi > hi) return false;
                             if (write) return true;   // ordered before this write (checked above)
                             return !r.write && r.stream == x.stream;
                           }),
            rec.end());
  rec.push_back({lo, hi, write, x.stream, x.seq, x.what});
}

template <class T>
T load_dev(Op& x, const T* p, const char* what) {
  touch(x, (uintptr_t)p, sizeof(T), false, what);
  T v{};
  Alloc* a = find_alloc((uintptr_t)p);
  if (a && !a->freed && (uintptr_t)p + sizeof(T) <= a->hi) std::memcpy(&v, p, sizeof(T));
  return v;
}

size_t span_words(uint64_t batch, uint64_t stride, uint64_t rows, uint64_t ld, uint64_t lanes) {
  if (!batch || !rows || !lanes) return 0;
  return (batch - 1) * stride + (rows - 1) * ld + lanes;
}

// ------------------------------------------------------------ kernel models
std::vector<int> template_ints(const std::string& name) {
  std::vector<int> v;
  const size_t a = name.find('<');
  if (a == std::string::npos) return v;
  const size_t b = name.find('>', a);
  std::string in = name.substr(a + 1, b - a - 1);
  size_t pos = 0;
  while (pos < in.size()) {
    size_t e = in.find(',', pos);
    if (e == std::string::npos) e = in.size();
    v.push_back(atoi(in.substr(pos, e - pos).c_str()));
    pos = e + 1;
  }
  return v;
}

void model_tw(Op& x, const uint32_t* tw, const uint32_t* twi) {
  touch(x, (uintptr_t)tw, 65536 * 4, false, "tw");
  touch(x, (uintptr_t)twi, 65536 * 4, false, "twi");
  touch(x, (uintptr_t)(tw + fntrs::kStageTwBase), fntrs::kStageTwWords * 4, false, "stage twiddles");
}

void model_encode(Op& x, const EncodeArgs& a, uint64_t items, uint64_t per_block) {
  if (!a.tiles || !a.cosets || items % per_block) {
    error(x.what + ": work items " + std::to_string(items) + " do not split into blocks");
    return;
  }
  const uint64_t batch = items / per_block;
  touch(x, (uintptr_t)a.src, span_words(batch, a.stride_src, a.k, a.ld_src, a.lanes) * 4, false, "src");
  const uint32_t rows = a.rows_out ? a.rows_out : a.n;
  touch(x, (uintptr_t)a.dst, span_words(batch, a.stride_dst, rows, a.ld_dst, a.lanes) * 4, true, "dst");
  model_tw(x, a.tw, a.twi);
}

void model_decode(Op& x, const DecodeArgs& a, uint64_t items, int D) {
  if (!a.tiles || items % a.tiles) {
    error(x.what + ": work items do not split into blocks");
    return;
  }
  const uint64_t batch = items / a.tiles;
  const uint32_t rows = a.full ? a.n : a.k;
  touch(x, (uintptr_t)a.recv, span_words(batch, a.stride_recv, rows, a.ld_recv, a.lanes) * 4, false, "recv");
  touch(x, (uintptr_t)a.dst, span_words(batch, a.stride_dst, a.k, a.ld_dst, a.lanes) * 4, true, "dst");
  if (a.wrb) {
    touch(x, (uintptr_t)a.wrb, (size_t)a.n * 8, false, "first-pass pairs");
  } else {
    touch(x, (uintptr_t)a.wfull, (size_t)a.n * 4, false, "wfull");
    if (!a.full && D >= 0) touch(x, (uintptr_t)a.ridx, (size_t)a.n * 4, false, "ridx");
  }
  if (D >= 0) touch(x, (uintptr_t)a.ahat_br, (size_t)(a.n >> D) * 4, false, "ahat_br");
  model_tw(x, a.tw, a.twi);
}

template <class Args, class F>
void model_table(Op& x, const JobTable<Args>& t, F per_job) {
  if (!t.njobs) {
    error(x.what + ": empty job table");
    return;
  }
  touch(x, (uintptr_t)t.start, (size_t)(t.njobs + 1) * 4, false, "job starts");
  touch(x, (uintptr_t)t.jobs, (size_t)t.njobs * sizeof(Args), false, "job table");
  std::vector<uint32_t> start(t.njobs + 1);
  for (uint32_t j = 0; j <= t.njobs; ++j) start[j] = load_dev(x, t.start + j, "job starts");
  if (start[0] != 0 || start[t.njobs] != t.total) error(x.what + ": job table does not cover the work items");
  for (uint32_t j = 0; j < t.njobs; ++j) {
    if (start[j + 1] < start[j]) {
      error(x.what + ": job starts not ascending");
      return;
    }
    const Args a = load_dev(x, t.jobs + j, "job table");
    per_job(a, (uint64_t)start[j + 1] - start[j]);
  }
}

void model_fourstep(Op& x, const std::string& base, const FourStepArgs& a, uint64_t grid) {
  if (!a.tiles || !a.subs || grid % ((uint64_t)a.tiles * a.subs)) {
    error(x.what + ": grid does not split into blocks");
    return;
  }
  const uint64_t batch = grid / ((uint64_t)a.tiles * a.subs);
  uint64_t rin = 0, rout = 0;
  if (base == "k4_enc1") { rin = a.k; rout = a.n; }
  else if (base == "k4_enc2") { rin = a.n; rout = a.rows_out ? a.rows_out : a.n; }
  else if (base == "k4_dec1") {
    rin = a.full ? a.n : a.k;
    rout = a.n;
    touch(x, (uintptr_t)a.wr, (size_t)a.n * 8, false, "weights and rows by sub-transform");
  } else if (base == "k4_dec2") { rin = a.n; rout = a.M; }
  else if (base == "k4_dec3") {
    rin = a.M;
    rout = a.M;
    touch(x, (uintptr_t)a.ahat_t, (size_t)a.M * 4, false, "ahat by sub-transform");
  } else if (base == "k4_dec4") { rin = a.M; rout = a.k; }
  else {
    error("no model of four-step kernel " + base);
    return;
  }
  // element (b, row, tile*T + l) lies at b*stride + tile*tstride + row*ld + l:
  // row-major buffers have tstride = T (the span of all lanes), tile-major
  // scratch has tstride = rows*T and holds whole tiles of T lanes
  constexpr uint64_t T = 32;
  auto span = [&](uint64_t stride, uint64_t tstride, uint64_t rows, uint64_t ld) -> size_t {
    if (tstride == T) return span_words(batch, stride, rows, ld, a.lanes);
    if (!batch || !rows) return 0;
    if (tstride < rows * ld) error(x.what + ": lane tiles of a tile-major buffer overlap");
    return (batch - 1) * stride + (uint64_t)(a.tiles - 1) * tstride + (rows - 1) * ld + T;
  };
  touch(x, (uintptr_t)a.in, span(a.stride_in, a.tstride_in, rin, a.ld_in) * 4, false, "in");
  touch(x, (uintptr_t)a.out, span(a.stride_out, a.tstride_out, rout, a.ld_out) * 4, true, "out");
  // a tile-major scratch buffer's escape bitmap: one bit per row of a tile
  if (a.tstride_in != T)
    touch(x, (uintptr_t)a.in + a.boff_in, (size_t)batch * a.tiles * (a.tstride_in / T) / 8, false, "escape bits in");
  if (a.tstride_out != T)
    touch(x, (uintptr_t)a.out + a.boff_out, (size_t)batch * a.tiles * (a.tstride_out / T) / 8, true, "escape bits out");
  model_tw(x, a.tw, a.twi);
  // split twiddles of the kernels that have them: a table of n (K1, encoder
  // pass A) or M (K2, K3) words
  if (base == "k4_dec1" || base == "k4_enc1")
    touch(x, (uintptr_t)a.twsplit, (size_t)a.n * 4, false, "split twiddles");
  if (base == "k4_dec2" || base == "k4_dec3")
    touch(x, (uintptr_t)a.twsplit, (size_t)a.M * 4, false, "split twiddles");
}

void model_locdesc(Op& x, const LocDesc& d) {
  const size_t n = d.n, kr = d.kr, kt = d.k, M = kr < n ? (size_t)1 << d.logm : 0;
  if (d.zin) touch(x, (uintptr_t)d.zin, kr * 4, false, "zin");   // null: positions passed by value
  struct {
    const void* p;
    size_t words;
    const char* name;
  } rw[] = {{d.pos, kr, "pos"},   {d.wfull, n, "wfull"}, {d.ridx, n, "ridx"},   {d.ahat_br, M, "ahat_br"},
            {d.ahat_s, M, "ahat_s"}, {d.A, kr + 1, "A"},  {d.w, kr, "w"},        {d.ahat, M, "ahat"},
            {d.t0, kt, "t0"},      {d.t1, kt, "t1"},      {d.spec, kt, "spec"}, {d.vals, n, "vals"}};
  for (auto& r : rw)
    if (r.p && r.words) touch(x, (uintptr_t)r.p, r.words * 4, true, r.name);
}

void model_loc_range(Op& x, const LocDesc* D, const uint32_t* start, uint32_t count, const uint32_t* tw) {
  if (start) touch(x, (uintptr_t)start, (size_t)(count + 1) * 4, false, "stage starts");
  touch(x, (uintptr_t)D, (size_t)count * sizeof(LocDesc), false, "descriptors");
  for (uint32_t i = 0; i < count; ++i) model_locdesc(x, load_dev(x, D + i, "descriptors"));
  if (tw) touch(x, (uintptr_t)tw, 65536 * 4, false, "tw");
}

// Builds the executing model of one launch from its arguments (copied now,
// as the launch does).
std::function<void(Op&)> kernel_model(const std::string& name, dim3 grid, void** args) {
  std::string base = name;
  for (size_t an; (an = base.find("(anonymous namespace)::")) != std::string::npos;)
    base.erase(an, std::strlen("(anonymous namespace)::"));
  const size_t par = base.find('(');
  if (par != std::string::npos) base = base.substr(0, par);
  const size_t lt = base.find('<');
  const std::string head = lt == std::string::npos ? base : base.substr(0, lt);
  const std::string fn = head.substr(head.rfind(':') + 1);
  const std::vector<int> tp = template_ints(base);
  const uint64_t g = (uint64_t)grid.x * grid.y * grid.z;
  if (fn == "k_enc" || fn == "k_enc_cos") {
    const EncodeArgs a = *(const EncodeArgs*)args[0];
    const bool cos = fn == "k_enc_cos";
    return [a, g, cos](Op& x) { model_encode(x, a, cos ? g * a.cosets : g, (uint64_t)a.tiles * a.cosets); };
  }
  if (fn == "k_enc_tab" || fn == "k_enc_cos_tab") {
    const JobTable<EncodeArgs> t = *(const JobTable<EncodeArgs>*)args[0];
    const bool cos = fn == "k_enc_cos_tab";   // a work item covers every coset of its tile
    return [t, cos](Op& x) {
      model_table(x, t, [&](const EncodeArgs& a, uint64_t items) {
        model_encode(x, a, cos ? items * a.cosets : items, (uint64_t)a.tiles * a.cosets);
      });
    };
  }
  if (fn == "k_dec") {
    const DecodeArgs a = *(const DecodeArgs*)args[0];
    const int D = tp.size() > 1 ? tp[1] : 0;
    return [a, g, D](Op& x) { model_decode(x, a, g, D); };
  }
  if (fn == "k_dec_tab" || fn == "k_dec_pipe") {
    const JobTable<DecodeArgs> t = *(const JobTable<DecodeArgs>*)args[0];
    const int D = tp.size() > 1 ? tp[1] : 0;
    DecodeArgs one{};
    if (fn == "k_dec_pipe") one = *(const DecodeArgs*)args[1];
    return [t, one, D](Op& x) {
      if (!t.jobs) {
        model_decode(x, one, t.total, D);
        return;
      }
      model_table(x, t, [&](const DecodeArgs& a, uint64_t items) { model_decode(x, a, items, D); });
    };
  }
  if (fn == "k_dec_pairs") {   // (wfull, ridx, wrb, n, logn, full)
    const uint32_t* wf = *(const uint32_t* const*)args[0];
    const uint32_t* ri = *(const uint32_t* const*)args[1];
    uint32_t* wrb = *(uint32_t* const*)args[2];
    const uint32_t n = *(const uint32_t*)args[3];
    const uint32_t full = *(const uint32_t*)args[5];
    return [wf, ri, wrb, n, full](Op& x) {
      touch(x, (uintptr_t)wf, (size_t)n * 4, false, "wfull");
      if (!full) touch(x, (uintptr_t)ri, (size_t)n * 4, false, "ridx");
      touch(x, (uintptr_t)wrb, (size_t)n * 8, true, "first-pass pairs");
    };
  }
  if (fn == "k_fs_prep") {   // zeroes up to three ranges of 16-byte vectors
    const fntrs::FsPrepArgs c = *(const fntrs::FsPrepArgs*)args[0];
    return [c](Op& x) {
      for (int j = 0; j < 3; ++j)
        if (c.words[j]) {
          if (c.words[j] % 4 || (uintptr_t)c.p[j] % 16) error(x.what + ": clear range is not whole 16-byte vectors");
          touch(x, (uintptr_t)c.p[j], c.words[j] * 4, true, "escape bits");
        }
      if (c.wr) {
        if ((uintptr_t)c.wr % 8) error(x.what + ": weight and row pairs are not 8-byte aligned");
        touch(x, (uintptr_t)c.wfull, (size_t)c.n * 4, false, "wfull");
        if (!c.full) touch(x, (uintptr_t)c.ridx, (size_t)c.n * 4, false, "ridx");
        touch(x, (uintptr_t)c.wr, (size_t)c.n * 8, true, "weights and rows by sub-transform");
      }
      if (c.ahat_t) {
        touch(x, (uintptr_t)c.ahat, (size_t)c.M * 4, false, "ahat");
        touch(x, (uintptr_t)c.ahat_t, (size_t)c.M * 4, true, "ahat by sub-transform");
      }
    };
  }
  if (fn.rfind("k4_", 0) == 0) {
    const FourStepArgs a = *(const FourStepArgs*)args[0];
    return [fn, a, g](Op& x) { model_fourstep(x, fn, a, g); };
  }
  if (fn == "k_locb_small1") {   // one pattern, descriptor and positions by value
    const fntrs::LocSmallOne a = *(const fntrs::LocSmallOne*)args[0];
    const uint32_t* tw = *(const uint32_t* const*)args[1];
    return [a, tw](Op& x) {
      model_locdesc(x, a.d);
      touch(x, (uintptr_t)tw, 65536 * 4, false, "tw");
    };
  }
  if (fn == "k_locb_small") {
    const LocDesc* D = *(const LocDesc* const*)args[0];
    const uint32_t* tw = *(const uint32_t* const*)args[1];
    return [D, g, tw](Op& x) { model_loc_range(x, D, nullptr, (uint32_t)g, tw); };
  }
  if (fn.rfind("k_locb_", 0) == 0) {
    const LocDesc* D = *(const LocDesc* const*)args[0];
    const uint32_t* start = *(const uint32_t* const*)args[1];
    const uint32_t count = *(const uint32_t*)args[2];
    return [D, start, count](Op& x) { model_loc_range(x, D, start, count, nullptr); };
  }
  if (fn == "k_loc_mul") {
    uint32_t* xp = *(uint32_t* const*)args[0];
    const uint32_t* yp = *(const uint32_t* const*)args[1];
    const uint32_t count = *(const uint32_t*)args[2];
    return [=](Op& x) {
      touch(x, (uintptr_t)yp, (size_t)count * 4, false, "y");
      touch(x, (uintptr_t)xp, (size_t)count * 4, true, "x");
    };
  }
  if (fn == "k_conv_mark") {   // workgroup b: positions [256 b, 256 b + 256)
    const uint32_t* zin = *(const uint32_t* const*)args[0];
    const uint32_t* bstart = *(const uint32_t* const*)args[1];
    uint32_t* ind = *(uint32_t* const*)args[2];
    uint32_t* pos = *(uint32_t* const*)args[3];
    uint32_t* ridx = *(uint32_t* const*)args[4];
    // tables read from pinned host memory: the bytes as of the launch
    auto pinned_copy = [](const void* p, size_t bytes) {
      Alloc* a = find_alloc((uintptr_t)p);
      std::shared_ptr<std::vector<uint8_t>> v;
      if (a && a->kind == 2 && (uintptr_t)p + bytes <= a->hi)
        v = std::make_shared<std::vector<uint8_t>>((const uint8_t*)p, (const uint8_t*)p + bytes);
      return v;
    };
    const auto sb = pinned_copy(bstart, ((size_t)g + 1) * 4);
    const auto sz = sb ? pinned_copy(zin, (size_t)bstart[g] * 4) : nullptr;
    return [=](Op& x) {
      const size_t n = (size_t)g * 256;
      touch(x, (uintptr_t)bstart, ((size_t)g + 1) * 4, false, "bstart");
      const uint32_t kr = bstart[g];   // the host table: every rank below n
      touch(x, (uintptr_t)zin, (size_t)kr * 4, false, "zin");
      if ((sb && std::memcmp(sb->data(), bstart, sb->size()) != 0) ||
          (sz && std::memcmp(sz->data(), zin, sz->size()) != 0))
        error("pinned staging overwritten by the host before its kernel ran (" + x.what + ")");
      touch(x, (uintptr_t)ind, n * 4, true, "ind");
      touch(x, (uintptr_t)pos, (size_t)kr * 4, true, "pos");
      touch(x, (uintptr_t)ridx, n * 4, true, "ridx");
    };
  }
  if (fn == "k_conv_mul") {
    const uint32_t* F = *(const uint32_t* const*)args[0];
    const uint32_t* T = *(const uint32_t* const*)args[1];
    uint32_t* P = *(uint32_t* const*)args[2];
    const uint32_t n = *(const uint32_t*)args[3];
    return [=](Op& x) {
      touch(x, (uintptr_t)F, (size_t)n * 4, false, "F");
      touch(x, (uintptr_t)T, (size_t)n * 64, false, "T");
      touch(x, (uintptr_t)P, (size_t)n * 64, true, "P");
    };
  }
  if (fn == "k_conv_finish") {
    const fntrs::ConvFinishArgs a = *(const fntrs::ConvFinishArgs*)args[0];
    return [=](Op& x) {
      const size_t n = (size_t)1 << a.logn, M = (size_t)1 << a.logm;
      touch(x, (uintptr_t)a.Q, n * 64, false, "Q");
      touch(x, (uintptr_t)a.ind, n * 4, false, "ind");
      touch(x, (uintptr_t)a.ridx, n * 4, false, "ridx");
      touch(x, (uintptr_t)a.tw, 65536 * 4, false, "tw");
      touch(x, (uintptr_t)a.w, (size_t)a.kr * 4, true, "w");
      touch(x, (uintptr_t)a.wfull, n * 4, true, "wfull");
      touch(x, (uintptr_t)a.ahat, M * 4, true, "ahat");
      touch(x, (uintptr_t)a.ahat_br, M * 4, true, "ahat_br");
      touch(x, (uintptr_t)a.ahat_s, M * 4, true, "ahat_s");
      touch(x, (uintptr_t)a.vals, n * 4, true, "vals");
    };
  }
  if (fn == "k_conv_coef") {
    const uint32_t* G = *(const uint32_t* const*)args[0];
    uint32_t* A = *(uint32_t* const*)args[1];
    const uint32_t kr = *(const uint32_t*)args[2];
    const int logn = *(const int*)args[3];
    return [=](Op& x) {
      touch(x, (uintptr_t)G, ((size_t)1 << logn) * 4, false, "G");
      touch(x, (uintptr_t)A, ((size_t)kr + 1) * 4, true, "A");
    };
  }
  if (fn == "k_loc_combine") {
    const uint32_t* F = *(const uint32_t* const*)args[0];
    const uint32_t* a = *(const uint32_t* const*)args[1];
    const uint32_t* b = *(const uint32_t* const*)args[2];
    uint32_t* out = *(uint32_t* const*)args[3];
    const uint32_t d = *(const uint32_t*)args[4];
    return [=](Op& x) {
      touch(x, (uintptr_t)F, (size_t)2 * d * 4, false, "F");
      touch(x, (uintptr_t)a, (size_t)d * 4, false, "a");
      touch(x, (uintptr_t)b, (size_t)d * 4, false, "b");
      touch(x, (uintptr_t)out, (size_t)2 * d * 4, true, "out");
    };
  }
  if (fn == "k_copy_rows") {
    const uint32_t* src = *(const uint32_t* const*)args[0];
    const uint64_t ss = *(const uint64_t*)args[1];
    uint32_t* dst = *(uint32_t* const*)args[2];
    const uint64_t sd = *(const uint64_t*)args[3];
    const uint32_t lanes = *(const uint32_t*)args[4], batch = *(const uint32_t*)args[5];
    return [=](Op& x) {
      touch(x, (uintptr_t)src, span_words(batch, ss, 1, 0, lanes) * 4, false, "src");
      touch(x, (uintptr_t)dst, span_words(batch, sd, 1, 0, lanes) * 4, true, "dst");
    };
  }
  if (fn == "k_gemm_modp") {
    const GemmArgs a = *(const GemmArgs*)args[0];
    const uint64_t batch = grid.z;
    return [a, batch](Op& x) {
      // row maps are read from the simulated memory; rows they name are touched one by one
      auto rows_of = [&](const uint32_t* map, uint32_t count, const char* what) {
        std::vector<uint32_t> r(count);
        if (map) touch(x, (uintptr_t)map, (size_t)count * 4, false, what);
        for (uint32_t i = 0; i < count; ++i) r[i] = map ? load_dev(x, map + i, what) : i;
        return r;
      };
      if (a.M) touch(x, (uintptr_t)a.M, ((size_t)(a.R - 1) * a.ldm + a.K) * 4, false, "M");
      else {
        if (a.pw) touch(x, (uintptr_t)a.pw, (size_t)a.R * 4, false, "pw");
        touch(x, (uintptr_t)a.tw, 65536 * 4, false, "tw");
      }
      for (uint32_t r : rows_of(a.xrow, a.K, "xrow"))
        for (uint64_t b = 0; b < batch; ++b)
          touch(x, (uintptr_t)(a.X + b * a.stride_x + (uint64_t)r * a.ld_x), (size_t)a.lanes * 4, false, "X row");
      for (uint32_t r : rows_of(a.yrow, a.R, "yrow"))
        for (uint64_t b = 0; b < batch; ++b)
          touch(x, (uintptr_t)(a.Y + b * a.stride_y + (uint64_t)r * a.ld_y), (size_t)a.lanes * 4, true, "Y row");
    };
  }
  if (fn == "k_inv_vandermonde") {
    const uint32_t* A = *(const uint32_t* const*)args[0];
    const uint32_t* w = *(const uint32_t* const*)args[1];
    const uint32_t* pos = *(const uint32_t* const*)args[2];
    const uint32_t* tw = *(const uint32_t* const*)args[3];
    const uint32_t* twi = *(const uint32_t* const*)args[4];
    const uint32_t k = *(const uint32_t*)args[6];
    uint32_t* W = *(uint32_t* const*)args[7];
    return [=](Op& x) {
      touch(x, (uintptr_t)A, (size_t)(k + 1) * 4, false, "A");
      touch(x, (uintptr_t)w, (size_t)k * 4, false, "w");
      touch(x, (uintptr_t)pos, (size_t)k * 4, false, "pos");
      model_tw(x, tw, twi);
      touch(x, (uintptr_t)W, (size_t)k * k * 4, true, "W");
    };
  }
  if (fn == "k_copy_rowmap") {
    const uint32_t* src = *(const uint32_t* const*)args[0];
    const uint64_t ld_s = *(const uint64_t*)args[1], st_s = *(const uint64_t*)args[2];
    const uint32_t* srow = *(const uint32_t* const*)args[3];
    uint32_t* dst = *(uint32_t* const*)args[4];
    const uint64_t ld_d = *(const uint64_t*)args[5], st_d = *(const uint64_t*)args[6];
    const uint32_t* drow = *(const uint32_t* const*)args[7];
    const uint32_t rows = *(const uint32_t*)args[8], lanes = *(const uint32_t*)args[9];
    const uint64_t batch = grid.z;
    return [=](Op& x) {
      for (uint32_t r = 0; r < rows; ++r) {
        const uint32_t rs = srow ? load_dev(x, srow + r, "srow") : r, rd = drow ? load_dev(x, drow + r, "drow") : r;
        for (uint64_t b = 0; b < batch; ++b) {
          touch(x, (uintptr_t)(src + b * st_s + (uint64_t)rs * ld_s), (size_t)lanes * 4, false, "src row");
          touch(x, (uintptr_t)(dst + b * st_d + (uint64_t)rd * ld_d), (size_t)lanes * 4, true, "dst row");
        }
      }
    };
  }
  return [name](Op&) { error("no model of kernel " + name); };
}

// ------------------------------------------------------------ the device
bool runnable(const Op& op) {
  State& st = S();
  for (size_t t = 0; t < op.clk.size(); ++t)
    if ((int)t != op.stream && st.streams[t].exec < op.clk[t]) return false;
  return true;
}

void run_front(int s) {
  State& st = S();
  std::unique_ptr<Op> op = std::move(st.streams[s].q.front());
  st.streams[s].q.pop_front();
  if (op->run) op->run(*op);
  st.streams[s].exec = op->seq;
  ++st.ops_run;
}

// Executes up to `max` runnable operations in random order; returns how many ran.
int step(int max) {
  State& st = S();
  int done = 0;
  while (done < max) {
    std::vector<int> ready;
    for (size_t s = 0; s < st.streams.size(); ++s)
      if (!st.streams[s].q.empty() && runnable(*st.streams[s].q.front())) ready.push_back((int)s);
    if (ready.empty()) break;
    run_front(ready[st.rng() % ready.size()]);
    ++done;
  }
  return done;
}

// Lets the device run a random amount after a host call.
void maybe_progress() {
  State& st = S();
  std::uniform_real_distribution<double> u(0, 1);
  if (u(st.rng) < st.lag) return;
  step(1 + (int)(st.rng() % 8));
}

bool pending_any() {
  for (auto& s : S().streams)
    if (!s.q.empty()) return true;
  return false;
}

// Runs until `done()` holds; a deadlock (nothing runnable) is an error.
template <class F>
void run_until(F done, const char* why) {
  while (!done()) {
    if (step(1) == 0) {
      error(std::string("deadlock while waiting for ") + why);
      return;
    }
  }
}

bool event_done(const Event& e) {
  State& st = S();
  for (size_t t = 0; t < e.clk.size(); ++t)
    if (st.streams[t].exec < e.clk[t]) return false;
  return true;
}

void drain_all() {
  run_until([] { return !pending_any(); }, "device synchronisation");
  State& st = S();
  for (size_t t = 0; t < st.streams.size(); ++t) {
    if (st.host.size() < st.streams.size()) st.host.resize(st.streams.size(), 0);
    st.host[t] = std::max(st.host[t], st.streams[t].exec);
  }
}

Op& enqueue(int s, std::string what, std::function<void(Op&)> run) {
  State& st = S();
  Stream& q = st.streams[s];
  auto op = std::make_unique<Op>();
  op->stream = s;
  op->seq = ++q.enq;
  op->clk = q.clk;
  join(op->clk, st.host);
  if (op->clk.size() <= (size_t)s) op->clk.resize(s + 1, 0);
  op->clk[s] = op->seq - 1;
  op->what = std::move(what);
  op->run = std::move(run);
  q.clk = op->clk;
  q.clk[s] = op->seq;
  Op& ref = *op;
  q.q.push_back(std::move(op));
  return ref;
}

std::string short_name(const std::string& n) { return n.size() > 90 ? n.substr(0, 90) + "..." : n; }

// An address in the simulated device memory (whether allocated or not).
bool in_device_space(uintptr_t p) {
  State& st = S();
  return p >= st.dev_end - (size_t(1) << 42) && p < st.dev_end;
}

}  // namespace

extern "C" {

// ------------------------------------------------------------ control
void fakehip_seed(uint64_t seed) { S().rng.seed(seed); }
void fakehip_set_lag(double lag) { S().lag = lag; }
void fakehip_drain() {
  std::lock_guard<std::mutex> lk(S().mu);
  drain_all();
}
int fakehip_errors() { return (int)S().errors.size(); }
const char* fakehip_error_text(int i) {
  auto& e = S().errors;
  return (i >= 0 && i < (int)e.size()) ? e[i].c_str() : "";
}
void fakehip_stats(uint64_t* ops, uint64_t* kernels, uint64_t* checks) {
  *ops = S().ops_run;
  *kernels = S().kernels_run;
  *checks = S().checks;
}
void fakehip_alloc_stats(uint64_t* malloc_calls, uint64_t* malloc_async_calls, uint64_t* wait_event_calls) {
  *malloc_calls = S().n_malloc;
  *malloc_async_calls = S().n_malloc_async;
  *wait_event_calls = S().n_wait_event;
}

// ------------------------------------------------------------ registration
void** __hipRegisterFatBinary(const void*) {
  static void* handle = nullptr;
  return &handle;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void* hostFunction, char* deviceFunction, const char*, unsigned int, uint3*,
                           uint3*, dim3*, dim3*, int*) {
  int st = 0;
  char* dem = abi::__cxa_demangle(deviceFunction, nullptr, nullptr, &st);
  S().kernels[hostFunction] = dem ? dem : deviceFunction;
  free(dem);
}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
  std::lock_guard<std::mutex> lk(S().mu);
  const uintptr_t p = dev_alloc(size, 3);
  S().symbols[var] = {p, size};
}
hipError_t hipGetSymbolAddress(void** devPtr, const void* symbol) {
  auto it = S().symbols.find(symbol);
  if (it == S().symbols.end()) return hipErrorInvalidSymbol;
  *devPtr = (void*)it->second.first;
  return hipSuccess;
}

// ------------------------------------------------------------ device and properties
hipError_t hipGetDeviceCount(int* n) {
  *n = 1;
  return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDevicePropertiesR0600(hipDeviceProp_tR0600* p, int) {
  std::memset(p, 0, sizeof *p);
  std::snprintf(p->name, sizeof p->name, "simulated gfx950");
  p->multiProcessorCount = 256;
  p->sharedMemPerBlock = 163840;
  p->warpSize = 64;
  p->maxThreadsPerBlock = 1024;
  return hipSuccess;
}
hipError_t hipDeviceGetDefaultMemPool(hipMemPool_t* pool, int) {
  static int dummy;
  *pool = (hipMemPool_t)&dummy;
  return hipSuccess;
}
hipError_t hipMemPoolGetAttribute(hipMemPool_t, hipMemPoolAttr, void* v) {
  *(uint64_t*)v = 0;
  return hipSuccess;
}
hipError_t hipMemPoolSetAttribute(hipMemPool_t, hipMemPoolAttr, void*) { return hipSuccess; }
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void*) {
  std::memset(a, 0, sizeof *a);
  a->maxThreadsPerBlock = 1024;
  return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* nb, const void*, int, size_t) {
  *nb = 1;
  return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "simulated error"; }

// ------------------------------------------------------------ memory
hipError_t hipMalloc(void** p, size_t bytes) {
  std::lock_guard<std::mutex> lk(S().mu);
  ++S().n_malloc;
  *p = (void*)dev_alloc(bytes, 0);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!p) return hipSuccess;
  drain_all();   // hipFree waits for the device
  auto it = S().allocs.find((uintptr_t)p);
  if (it == S().allocs.end() || it->second.freed || it->second.kind == 2) {
    error("hipFree of a pointer that is not a live device allocation: " + hexs((uintptr_t)p));
    return hipErrorInvalidValue;
  }
  it->second.freed = true;
  it->second.rec.clear();
  return hipSuccess;
}
hipError_t hipMallocAsync(void** p, size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  ++S().n_malloc_async;
  const uintptr_t a = dev_alloc(bytes, 1);
  if (!a) return hipErrorOutOfMemory;
  Op& op = enqueue(sid(s), "hipMallocAsync", nullptr);
  Alloc& al = S().allocs[a];
  al.alloc_stream = op.stream;
  al.alloc_seq = op.seq;
  *p = (void*)a;
  maybe_progress();
  return hipSuccess;
}
hipError_t hipFreeAsync(void* p, hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  auto it = S().allocs.find((uintptr_t)p);
  if (it == S().allocs.end() || it->second.kind != 1) {
    error("hipFreeAsync of a pointer that is not a stream-ordered allocation: " + hexs((uintptr_t)p));
    return hipErrorInvalidValue;
  }
  const uintptr_t key = (uintptr_t)p;
  enqueue(sid(s), "hipFreeAsync", [key](Op& x) {
    Alloc& a = S().allocs[key];
    if (a.freed) {
      error("double stream-ordered free");
      return;
    }
    for (const Record& r : a.rec)
      if (!hb(x, r.stream, r.seq))
        error("stream-ordered free on stream " + std::to_string(x.stream) + " is not ordered after " + r.what +
              " (stream " + std::to_string(r.stream) + "), which used the memory");
    a.freed = true;
    a.rec.clear();
  });
  maybe_progress();
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned int) {
  std::lock_guard<std::mutex> lk(S().mu);
  void* q = nullptr;
  if (posix_memalign(&q, 4096, std::max<size_t>(bytes, 1))) return hipErrorOutOfMemory;
  Alloc a;
  a.lo = (uintptr_t)q;
  a.hi = a.lo + bytes;
  a.kind = 2;
  S().allocs[a.lo] = a;
  *p = q;
  return hipSuccess;
}
// Pinned host memory is read by kernels at its own address.
hipError_t hipHostGetDevicePointer(void** d, void* h, unsigned int) {
  std::lock_guard<std::mutex> lk(S().mu);
  Alloc* a = find_alloc((uintptr_t)h);
  if (!d || !a || a->kind != 2) return hipErrorInvalidValue;
  *d = h;
  return hipSuccess;
}
hipError_t hipHostFree(void* p) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!p) return hipSuccess;
  drain_all();
  auto it = S().allocs.find((uintptr_t)p);
  if (it == S().allocs.end() || it->second.kind != 2) {
    error("hipHostFree of a pointer that is not pinned host memory");
    return hipErrorInvalidValue;
  }
  S().allocs.erase(it);
  free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  const uintptr_t d = (uintptr_t)dst, so = (uintptr_t)src;
  Alloc* sa = find_alloc(so);
  const bool src_tracked = sa != nullptr || in_device_space(so);
  const bool src_pinned = sa && sa->kind == 2;
  const bool dst_tracked = find_alloc(d) != nullptr || in_device_space(d);
  std::shared_ptr<std::vector<uint8_t>> snap;
  if (!src_tracked || src_pinned) {   // host source: the bytes as of now
    snap = std::make_shared<std::vector<uint8_t>>((const uint8_t*)src, (const uint8_t*)src + bytes);
  }
  enqueue(sid(s), "hipMemcpyAsync", [=](Op& x) {
    if (src_tracked) touch(x, so, bytes, false, "copy source");
    if (dst_tracked) touch(x, d, bytes, true, "copy destination");
    if (src_pinned && std::memcmp(snap->data(), (const void*)so, bytes) != 0)
      error("pinned staging overwritten by the host before its copy ran (" + std::to_string(bytes) + " bytes)");
    Alloc* da = find_alloc(d);
    const bool src_ok = !src_tracked || src_pinned || (sa && !sa->freed && so + bytes <= sa->hi);
    if (!dst_tracked || (da && !da->freed && d + bytes <= da->hi)) {
      if (snap) std::memcpy((void*)d, snap->data(), bytes);
      else if (src_ok) std::memmove((void*)d, (const void*)so, bytes);
    }
  });
  maybe_progress();
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  {
    std::lock_guard<std::mutex> lk(S().mu);
    run_until([] { return S().streams[0].q.empty(); }, "hipMemcpy on the null stream");
  }
  const hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, nullptr);
  std::lock_guard<std::mutex> lk(S().mu);
  run_until([] { return S().streams[0].q.empty(); }, "hipMemcpy");
  join(S().host, S().streams[0].clk);
  return e;
}
hipError_t hipMemsetAsync(void* p, int v, size_t bytes, hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  const uintptr_t d = (uintptr_t)p;
  enqueue(sid(s), "hipMemsetAsync", [=](Op& x) {
    touch(x, d, bytes, true, "memset");
    Alloc* a = find_alloc(d);
    if (a && !a->freed && d + bytes <= a->hi) std::memset((void*)d, v, bytes);
  });
  maybe_progress();
  return hipSuccess;
}

// ------------------------------------------------------------ streams and events
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  std::lock_guard<std::mutex> lk(S().mu);
  State& st = S();
  st.streams.emplace_back();
  *s = new ihipStream_t{(int)st.streams.size() - 1};
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  if (!s) return hipErrorInvalidValue;
  S().streams[s->id].destroyed = true;   // its queue still drains
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  const int id = sid(s);
  run_until([id] { return S().streams[id].q.empty(); }, "stream synchronisation");
  join(S().host, S().streams[id].clk);
  return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
  std::lock_guard<std::mutex> lk(S().mu);
  drain_all();
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  std::lock_guard<std::mutex> lk(S().mu);
  ++S().n_wait_event;
  if (!e) return hipErrorInvalidValue;
  const Event& ev = S().events[e->id];
  if (ev.recorded) join(S().streams[sid(s)].clk, ev.clk);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int) {
  std::lock_guard<std::mutex> lk(S().mu);
  S().events.emplace_back();
  *e = new ihipEvent_t{(int)S().events.size() - 1};
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  Event& ev = S().events[e->id];
  ev.clk = S().streams[sid(s)].clk;
  ev.recorded = true;
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(S().mu);
  maybe_progress();
  Event& ev = S().events[e->id];
  if (!ev.recorded) return hipSuccess;
  if (!event_done(ev)) return hipErrorNotReady;
  join(S().host, ev.clk);
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(S().mu);
  Event& ev = S().events[e->id];
  if (!ev.recorded) return hipSuccess;
  run_until([&ev] { return event_done(ev); }, "an event");
  join(S().host, ev.clk);
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f;
  return hipSuccess;
}

// ------------------------------------------------------------ launches
hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t shm, hipStream_t s) {
  S().cfg.push_back({g, b, shm, s});
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* shm, hipStream_t* s) {
  auto& c = S().cfg;
  if (c.empty()) return hipErrorInvalidConfiguration;
  *g = c.back().g;
  *b = c.back().b;
  *shm = c.back().shm;
  *s = c.back().s;
  c.pop_back();
  return hipSuccess;
}
hipError_t hipLaunchKernel(const void* f, dim3 grid, dim3 block, void** args, size_t, hipStream_t s) {
  std::lock_guard<std::mutex> lk(S().mu);
  auto it = S().kernels.find(f);
  const std::string name = it == S().kernels.end() ? std::string("<unregistered kernel>") : it->second;
  if ((uint64_t)grid.x * grid.y * grid.z == 0 || block.x == 0) error("empty launch of " + name);
  auto model = kernel_model(name, grid, args);
  enqueue(sid(s), short_name(name), [model](Op& x) {
    ++S().kernels_run;
    model(x);
  });
  maybe_progress();
  return hipSuccess;
}

// ------------------------------------------------------------ graphs (not simulated)
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = nullptr;
  return hipErrorNotSupported;
}
hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  return hipErrorNotSupported;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }

}  // extern "C"
