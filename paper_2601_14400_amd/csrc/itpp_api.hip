// Host runtime and C ABI of the ITPP engine (see include/itpp.h).
//
// The host owns the schedule and the bit permutation ("rep") of the stored
// keys.  For every elementary gate it computes cosh/sinh of the angle
// theta = alpha_k * m * dtau (Algorithm 1, Eq. ITPP_PropRules), the rep
// positions of the bits the gate tests and flips, and the move of the next
// gate's flip bits to the top of the rep; it then enqueues the gate kernel
// and the selection kernels on the context's stream without waiting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/itpp.h"
#include "itpp_internal.h"
#include "itpp_readout.h"

using namespace itpp;

namespace {

struct TermInfo {
  std::vector<uint64_t> x, z;  // canonical words
  double alpha = 0.0;
  bool identity = true;
  std::vector<int> F;      // canonical bits flipped (x_j -> j, z_j -> n + j), ascending
  std::vector<int> cbits;  // canonical bits whose parity marks anticommutation
  int nsup = 0;
  int sup[2] = {0, 0};
  int qx[2] = {0, 0}, qz[2] = {0, 0};
  int aQ = 0;
};

// Host state before one enqueued gate (to redo a speculative gate).
struct HostSnap {
  std::vector<int> pos;
  int cur, par, gpos;
  uint64_t serial;
  size_t ev_used;
};

// A stored state in the packed layout (regions back to back), with the
// host data needed to continue the schedule from it.
struct Snapshot {
  void* owned = nullptr;  // allocation owned by the snapshot (forward checkpoints), else arena memory
  Side side{};
  Plan* plan = nullptr;
  Filter* filt = nullptr;
  uint64_t count = 0;
  std::vector<int> pos;
  int gpos = 0;
  int64_t gate = 0;  // gates applied before this state since the last reset
};

}  // namespace

struct itpp_ctx_s {
  itpp_config cfg{};
  int n = 0, W = 1, NW = 2, nbits = 2;
  int f32 = 0, coef_bytes = 8;  // stored coefficient type: binary32 or binary64
  int shape = 0;                // ITPP_OPT_GATE_SHAPE (0, 1, 2, or kShapeAuto)
  uint64_t state_hint = 1;      // stored strings at the last host synchronisation (automatic shape)
  // device memory: own allocations, or a slice of a batch arena
  uint8_t* arena = nullptr;
  uint64_t arena_size = 0, arena_top = 0;
  bool measure = false;          // only add up the bytes the buffers need
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  int cus = 256;
  uint64_t cap = 0;  // elements per side
  Side side[2]{};
  Plan* plan = nullptr;    // [2]
  Filter* filt = nullptr;  // [2]
  Ctl* ctl = nullptr;
  TileStatus* status = nullptr;
  uint64_t status_cap = 0;
  uint64_t* part = nullptr;  // merge-path boundaries (2 words each)
  SelBuf sel{};
  double* d_result = nullptr;
  unsigned long long* d_count = nullptr;  // strings written by itpp_export_device
  std::vector<void*> allocs;
  // model
  std::vector<TermInfo> terms;
  std::vector<int> sched_term;
  std::vector<double> sched_mult;
  std::vector<int> glist;  // schedule positions of non-identity gates
  // state
  std::vector<int> pos;  // canonical bit -> rep position of the stored state
  int cur = 0;           // side holding the stored state
  int gpos = 0;          // index in glist of the next gate to apply
  int par = 0;           // plan/filter slot describing the stored state
  bool ready = false;
  uint64_t serial = 0;  // the device's gate serial of the next enqueued gate (mirror)
  bool speculate = true;
  bool real_time = false;       // gates follow the real-time rule (ITPP_OPT_REAL_TIME)
  double spec_mult = 0.98;
  int64_t retries_total = 0;
  std::string err;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;  // pool: 3 events per timed gate
  size_t ev_used = 0;
  double t_gate_ms = 0.0, t_sel_ms = 0.0, t_alg_bytes = 0.0;
  int64_t t_gates = 0;
  // reverse sweep
  int32_t ckpt_every = 0;       // Trotter steps between forward checkpoints (0: off)
  int64_t adj_workspace = 0;    // bytes for the reverse sweep's snapshots (0: automatic)
  int64_t fwd_gates = 0;        // gates applied since the last reset
  double fwd_dtau = 0.0;        // their common dtau
  bool fwd_valid = true;        // false once the gates since reset cannot be replayed
  std::vector<Snapshot> ckpts;  // forward checkpoints
  // Recorded graph of one Trotter step.  The bit order of the stored keys
  // at the start of a step is the same from the second step on (every step
  // moves the same bits in the same order), so the launches of a step,
  // whose arguments depend only on that order, dtau and the options, are
  // recorded once and replayed.
  bool graphs = true;                // ITPP_OPT_GRAPHS
  int grid_div = 1;                  // ITPP_OPT_GRID_DIV: gate kernel grid = resident workgroups / grid_div
  int max_weight = 0;                // ITPP_OPT_MAX_WEIGHT: Pauli-weight cutoff (0: none)
  hipGraphExec_t step_exec = nullptr;
  std::vector<int> step_pos;         // bit order at the start of the recorded step
  int step_cur = -1, step_par = -1;  // ping-pong slots it starts from
  double step_dtau = 0.0;
  int step_shape = -1;               // gate kernel shape it was recorded with
  std::vector<HostSnap> step_snaps;  // host state before each of its gates (serial relative)
  std::vector<int> last_step_pos;    // bit order at the start of the previous step
  int64_t graph_steps = 0;           // steps run as graph replays (statistics)
  int short_batches = 0;             // batches left at kSyncAfterHalt gates
  // The null stream cannot be captured: with cfg.stream == NULL the gates
  // run on a private non-blocking stream joined to the null stream by events
  // before and after (so they stay ordered with the caller's work).
  hipStream_t gate_stream = nullptr;
  hipEvent_t join_in = nullptr, join_out = nullptr;
};

namespace {

const char* kVersion = "itpp gfx950 merge-join engine 0.2";
// Host synchronisation period (gates) for the speculation check.
constexpr int64_t kSyncEvery = 512;
// ITPP_OPT_GATE_SHAPE 3 (the default): shape 2, the 256-thread layer kernel,
// while the stored state holds at most kAutoShapeMaxStrings strings, shape 1
// above.  Measured on one MI355X (TFIM chains, whole gates per second), the
// layer kernel is ahead up to 2^18 strings and behind from 2^20 on, for one-
// and two-word keys alike.
constexpr int kShapeAuto = 3;
constexpr uint64_t kAutoShapeMaxStrings = 1ull << 19;
// After a speculative gate had to be redone, the next few batches are short:
// a redone gate turns the rest of its batch into launches that return at
// once, and failures come in runs (when the cap starts to bind).
constexpr int64_t kSyncAfterHalt = 48;
constexpr int kShortBatchesAfterHalt = 8;
thread_local std::string g_create_error = "no error";

// Device scratch of itpp_expect_squared_noalloc: the observable words and
// weights it stages, the tables built from them, the per-block partial sums
// and the two results.  One copy per GPU, shared by every call on that GPU.
constexpr int32_t kSqMaxStrings = 4096;   // observable strings per call
constexpr int64_t kSqMaxSupport = 65536;  // non-identity sites summed over the strings
constexpr int kSqMaxGrid = 4096;          // blocks of the squared-state kernel
constexpr uint64_t sq_align(uint64_t b) { return (b + 255) & ~255ull; }
constexpr uint64_t kSqOffX = 0;
constexpr uint64_t kSqOffZ = kSqOffX + sq_align(8ull * kMaxWords * kSqMaxStrings);
constexpr uint64_t kSqOffOc = kSqOffZ + sq_align(8ull * kMaxWords * kSqMaxStrings);
constexpr uint64_t kSqOffQ = kSqOffOc + sq_align(8ull * kSqMaxStrings);
constexpr uint64_t kSqOffC = kSqOffQ + sq_align(8ull * kMaxKeyWords * kSqMaxStrings);
constexpr uint64_t kSqOffSupOff = kSqOffC + sq_align(8ull * kMaxKeyWords * kSqMaxStrings);
constexpr uint64_t kSqOffSupPos = kSqOffSupOff + sq_align(4ull * (kSqMaxStrings + 1));
constexpr uint64_t kSqOffSupQ = kSqOffSupPos + sq_align(8ull * kSqMaxSupport);
constexpr uint64_t kSqOffAq = kSqOffSupQ + sq_align(4ull * kSqMaxSupport);
constexpr uint64_t kSqOffCoef = kSqOffAq + sq_align(4ull * kSqMaxStrings);
constexpr uint64_t kSqOffPart = kSqOffCoef + sq_align(8ull * kSqMaxStrings);
constexpr uint64_t kSqOffOut = kSqOffPart + sq_align(32ull * kSqMaxGrid);
constexpr uint64_t kSqScratchBytes = kSqOffOut + 256;
static_assert(kSqScratchBytes <= (2ull << 20), "squared-state scratch stays below 2 MiB");

// In host code `scratch` only names the symbol; its device address on each
// GPU comes from hipGetSymbolAddress (scratch_address).
static __device__ __align__(256) unsigned char scratch[kSqScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on device dev, looked up once per device with
// that device current.
hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) {
      const hipError_t r = hipSetDevice(cur);
      if (e == hipSuccess) e = r;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

itpp_status create_fail(itpp_status s, const std::string& m) {
  g_create_error = m;
  return s;
}

itpp_status fail(itpp_ctx c, itpp_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

itpp_status hip_fail(itpp_ctx c, hipError_t e, const char* where) {
  return fail(c, ITPP_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                              \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

// Device memory owned by one API call; freed on every return path (hipFree
// waits for the work still using it).
struct DevBuf {
  void* p = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes); }
  template <typename T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

void move_top(std::vector<int>& pos, int cb, int nbits, int* old_pos) {
  const int p = pos[cb];
  if (old_pos) *old_pos = p;
  for (auto& q : pos)
    if (q > p) --q;
  pos[cb] = nbits - 1;
}

int popcount_words(const std::vector<uint64_t>& v) {
  int s = 0;
  for (auto w : v) s += __builtin_popcountll(w);
  return s;
}

void free_all(itpp_ctx c) {
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->ev_used = 0;
}

hipError_t next_event(itpp_ctx c, hipEvent_t* e) {
  if (c->ev_used == c->ev.size()) {
    hipEvent_t x;
    hipError_t r = hipEventCreate(&x);
    if (r != hipSuccess) return r;
    c->ev.push_back(x);
  }
  *e = c->ev[c->ev_used++];
  return hipSuccess;
}

// Sum the elapsed times of the recorded event triples and recycle the pool.
hipError_t drain_events(itpp_ctx c) {
  if (c->ev_used == 0) return hipSuccess;
  hipError_t r = hipStreamSynchronize(c->stream);
  if (r != hipSuccess) return r;
  for (size_t i = 0; i + 2 < c->ev_used; i += 3) {
    float a = 0.f, b = 0.f;
    r = hipEventElapsedTime(&a, c->ev[i], c->ev[i + 1]);
    if (r != hipSuccess) return r;
    r = hipEventElapsedTime(&b, c->ev[i + 1], c->ev[i + 2]);
    if (r != hipSuccess) return r;
    c->t_gate_ms += a;
    c->t_sel_ms += b;
    c->t_gates += 1;
  }
  c->ev_used = 0;
  return hipSuccess;
}

template <typename T>
hipError_t dalloc(itpp_ctx c, T** p, size_t count) {
  const uint64_t bytes = ((std::max<size_t>(count, 1) * sizeof(T)) + 255) & ~(uint64_t)255;
  if (c->measure) {
    c->arena_top += bytes;
    *p = nullptr;
    return hipSuccess;
  }
  if (c->arena) {
    if (c->arena_top + bytes > c->arena_size) return hipErrorOutOfMemory;
    *p = reinterpret_cast<T*>(c->arena + c->arena_top);
    c->arena_top += bytes;
    return hipSuccess;
  }
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e == hipSuccess) {
    c->allocs.push_back(q);
    *p = static_cast<T*>(q);
  }
  return e;
}

void free_ckpts(itpp_ctx c) {
  for (Snapshot& s : c->ckpts)
    if (s.owned) (void)hipFree(s.owned);
  c->ckpts.clear();
}

static_assert(sizeof(Plan) <= 512 && sizeof(Filter) <= 512, "snapshot header layout");

// Bytes of a packed snapshot of `count` elements (plan and filter first).
uint64_t snapshot_bytes(itpp_ctx c, uint64_t count) {
  const uint64_t head = 1024;
  const uint64_t words = ((count * 8 + 255) / 256) * 256;
  const uint64_t cb = ((count * (uint64_t)c->coef_bytes + 255) / 256) * 256;
  return head + (uint64_t)c->NW * words + cb;
}

// Element count of the stored state (host read of its plan).
hipError_t state_count(itpp_ctx c, uint64_t* out) {
  Plan p{};
  hipError_t e = hipMemcpyAsync(&p, c->plan + c->par, sizeof(Plan), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  uint64_t n = 0;
  for (int a = 0; a < (1 << p.wc); ++a)
    for (int b = 0; b < (1 << p.we); ++b) n += p.cnt[a][b];
  *out = n;
  return hipSuccess;
}

// Pack the stored state into `mem` (snapshot_bytes(count) bytes).
hipError_t write_snapshot(itpp_ctx c, Snapshot& s, void* mem, uint64_t count) {
  uint8_t* m = static_cast<uint8_t*>(mem);
  s.plan = reinterpret_cast<Plan*>(m);
  s.filt = reinterpret_cast<Filter*>(m + 512);
  s.count = count;
  uint8_t* q = m + 1024;
  const uint64_t words = ((count * 8 + 255) / 256) * 256;
  for (int w = 0; w < kMaxKeyWords; ++w) s.side.kw[w] = nullptr;
  for (int w = 0; w < c->NW; ++w) {
    s.side.kw[w] = reinterpret_cast<uint64_t*>(q);
    q += words;
  }
  s.side.coef = q;
  s.pos = c->pos;
  s.gpos = c->gpos;
  s.gate = c->fwd_gates;
  hipError_t e = launch_pack(c->NW, c->f32, c->side[c->cur], c->plan + c->par, s.side, s.plan, c->cus * 4,
                             c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s.filt, c->filt + c->par, sizeof(Filter), hipMemcpyDeviceToDevice, c->stream);
  return e;
}

// Make a snapshot the stored state again.
hipError_t restore_snapshot(itpp_ctx c, const Snapshot& s) {
  hipError_t e = hipSuccess;
  for (int w = 0; w < c->NW && e == hipSuccess; ++w)
    if (s.count) e = hipMemcpyAsync(c->side[c->cur].kw[w], s.side.kw[w], s.count * 8, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && s.count)
    e = hipMemcpyAsync(c->side[c->cur].coef, s.side.coef, s.count * (uint64_t)c->coef_bytes, hipMemcpyDeviceToDevice,
                       c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->plan + c->par, s.plan, sizeof(Plan), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->filt + c->par, s.filt, sizeof(Filter), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = launch_prepare(c->plan + (c->par ^ 1), c->ctl, c->stream);
  c->pos = s.pos;
  c->gpos = s.gpos;
  c->fwd_gates = s.gate;
  return e;
}

// Initial rep: identity permutation with the first gate's flip bits on top.
void initial_rep(itpp_ctx c, std::vector<int>& pos) {
  pos.resize(c->nbits);
  for (int i = 0; i < c->nbits; ++i) pos[i] = i;
  if (!c->glist.empty()) {
    const TermInfo& t = c->terms[c->sched_term[c->glist[0]]];
    for (int b : t.F) move_top(pos, b, c->nbits, nullptr);
  }
}

void reset_rep(itpp_ctx c) { initial_rep(c, c->pos); }

itpp_status do_reset(itpp_ctx c) {
  reset_rep(c);
  free_ckpts(c);
  c->fwd_gates = 0;
  c->fwd_dtau = 0.0;
  c->fwd_valid = true;
  int w0 = 0;
  if (!c->glist.empty()) w0 = (int)c->terms[c->sched_term[c->glist[0]]].F.size();
  c->cur = 0;
  c->par = 0;
  c->gpos = 0;
  c->state_hint = 1;
  HIP_TRY(c, launch_init(c->NW, c->f32, c->side[0], c->plan + 0, c->filt + 0, c->ctl, w0, c->stream));
  c->ready = true;
  return ITPP_OK;
}

itpp_status check_error(itpp_ctx c) {
  Ctl h{};
  HIP_TRY(c, hipMemcpyAsync(&h, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  switch (h.error) {
    case kErrNone:
      return ITPP_OK;
    case kErrNumeric:
      c->ready = false;
      return fail(c, ITPP_ERR_NUMERIC, "identity coefficient not finite or not positive; reset required");
    case kErrCap:
      c->ready = false;
      return fail(c, ITPP_ERR_CAP, "more than max_terms strings survived the threshold (ITPP_CAP_FAIL); reset required");
    case kErrPhase:
      c->ready = false;
      return fail(c, ITPP_ERR_DEVICE, "internal error: imaginary phase for commuting strings");
    case kErrSpin:
      c->ready = false;
      return fail(c, ITPP_ERR_DEVICE, "internal error: look-back wait exceeded its bound");
    default:
      c->ready = false;
      return fail(c, ITPP_ERR_DEVICE, "internal error: device buffer bound exceeded");
  }
}

}  // namespace

extern "C" {

const char* itpp_version(void) { return kVersion; }

const char* itpp_last_error(itpp_ctx ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->err.c_str();
}

}  // extern "C"

namespace {

itpp_status check_config(const itpp_config* cfg) {
  if (cfg->n_qubits < 1 || cfg->n_qubits > 64 * kMaxWords)
    return create_fail(ITPP_ERR_ARG, "n_qubits must be in 1..128");
  if (!(cfg->threshold >= 0.0) || !std::isfinite(cfg->threshold) || cfg->threshold >= 1.0)
    return create_fail(ITPP_ERR_ARG, "threshold must be finite, >= 0 and < 1");
  if (cfg->max_terms < 1) return create_fail(ITPP_ERR_ARG, "max_terms must be >= 1");
  if (cfg->precision != ITPP_F64 && cfg->precision != ITPP_F32)
    return create_fail(ITPP_ERR_ARG, "precision must be ITPP_F64 or ITPP_F32");
  if (cfg->cap_policy != ITPP_CAP_TOPK && cfg->cap_policy != ITPP_CAP_FAIL)
    return create_fail(ITPP_ERR_ARG, "unknown cap policy");
  return ITPP_OK;
}

itpp_status device_props(int* dev, hipDeviceProp_t* prop) {
  hipError_t he = hipGetDevice(dev);
  if (he != hipSuccess) return create_fail(ITPP_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(he));
  he = hipGetDeviceProperties(prop, *dev);
  if (he != hipSuccess)
    return create_fail(ITPP_ERR_DEVICE, std::string("hipGetDeviceProperties: ") + hipGetErrorString(he));
  if (std::string(prop->gcnArchName).rfind("gfx950", 0) != 0)
    return create_fail(ITPP_ERR_DEVICE, std::string("device is ") + prop->gcnArchName + ", not gfx950");
  return ITPP_OK;
}

// Create a context.  arena != NULL: its buffers are carved from
// [arena, arena + arena_size); measured != NULL: only return the bytes needed.
itpp_status create_impl(const itpp_config* cfg, int dev, const hipDeviceProp_t& prop, uint8_t* arena,
                        uint64_t arena_size, uint64_t* measured, itpp_ctx* out) {
  if (!measured) {
    void* sp = nullptr;
    const hipError_t se = scratch_address(dev, &sp);
    if (se != hipSuccess) return create_fail(ITPP_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(se));
  }
  itpp_ctx c = new (std::nothrow) itpp_ctx_s;
  if (!c) return ITPP_ERR_OOM;
  c->cfg = *cfg;
  c->n = cfg->n_qubits;
  c->W = (c->n + 63) / 64;
  c->NW = 2 * c->W;
  c->nbits = 2 * c->n;
  c->f32 = cfg->precision == ITPP_F32 ? 1 : 0;
  c->coef_bytes = c->f32 ? 4 : 8;
  c->shape = kShapeAuto;
  c->stream = static_cast<hipStream_t>(cfg->stream);
  c->device = dev;
  c->cus = prop.multiProcessorCount;
  c->arena = arena;
  c->arena_size = arena_size;
  c->measure = measured != nullptr;
  // every stored string comes from at most two outputs of a survivor and the
  // next gate's regions reserve twice the stored count: 4 K elements per side
  uint64_t kmax = (uint64_t)cfg->max_terms;
  if (c->n <= 30) kmax = std::min<uint64_t>(kmax, 1ull << (2 * c->n));
  c->cap = 4 * kmax + 64;
  const uint64_t elem_bytes = (uint64_t)c->NW * 8 + (uint64_t)c->coef_bytes;
  const int tile = gate_min_tile(c->NW);
  c->status_cap = c->cap / (uint64_t)tile + 16;
  const uint64_t sel_cap = 2 * kmax + 64;
  const uint64_t bytes = 2 * c->cap * elem_bytes + c->status_cap * kStatusWords * sizeof(TileStatus) +
                         sel_cap * (16 + 8 * (uint64_t)c->NW) + 4096;
  if (cfg->device_bytes_limit > 0 && bytes > (uint64_t)cfg->device_bytes_limit) {
    delete c;
    return create_fail(ITPP_ERR_OOM, "state buffers exceed device_bytes_limit");
  }
  bool ok = true;
  for (int s = 0; s < 2 && ok; ++s) {
    for (int q = 0; q < c->NW && ok; ++q) ok = dalloc(c, &c->side[s].kw[q], c->cap) == hipSuccess;
    if (ok) {
      uint8_t* cb = nullptr;
      ok = dalloc(c, &cb, c->cap * (uint64_t)c->coef_bytes) == hipSuccess;
      c->side[s].coef = cb;
    }
  }
  if (ok) ok = dalloc(c, &c->plan, 2) == hipSuccess;
  if (ok) ok = dalloc(c, &c->filt, 2) == hipSuccess;
  if (ok) ok = dalloc(c, &c->ctl, 1) == hipSuccess;
  if (ok) ok = dalloc(c, &c->status, c->status_cap * kStatusWords) == hipSuccess;
  if (ok) ok = dalloc(c, &c->part, 2 * (c->status_cap + kMaxClasses + 4)) == hipSuccess;
  if (ok) ok = dalloc(c, &c->sel.cand_bits, sel_cap) == hipSuccess;
  if (ok) ok = dalloc(c, &c->sel.cand_idx, sel_cap) == hipSuccess;
  if (ok) ok = dalloc(c, &c->sel.tie_keys, sel_cap * c->NW) == hipSuccess;
  if (ok) ok = dalloc(c, &c->d_result, 4) == hipSuccess;
  if (ok) ok = dalloc(c, &c->d_count, 1) == hipSuccess;
  if (measured) {
    *measured = c->arena_top;
    delete c;
    return ITPP_OK;
  }
  if (!ok) {
    (void)hipGetLastError();
    free_all(c);
    delete c;
    return create_fail(ITPP_ERR_OOM, "device memory for the state buffers is not available");
  }
  c->sel.cap = sel_cap;
  hipError_t he = hipMemsetAsync(c->status, 0, c->status_cap * kStatusWords * sizeof(TileStatus), c->stream);
  if (he == hipSuccess) he = hipMemsetAsync(c->plan, 0, 2 * sizeof(Plan), c->stream);
  if (he != hipSuccess) {
    free_all(c);
    delete c;
    return create_fail(ITPP_ERR_DEVICE, std::string("hipMemsetAsync: ") + hipGetErrorString(he));
  }
  if (do_reset(c) != ITPP_OK) {
    std::string m = c->err;
    free_all(c);
    delete c;
    return create_fail(ITPP_ERR_DEVICE, "initial state: " + m);
  }
  *out = c;
  return ITPP_OK;
}

}  // namespace

static void drop_step_graph(itpp_ctx c);

extern "C" {

itpp_status itpp_create(const itpp_config* cfg, itpp_ctx* out) {
  if (!cfg || !out) return create_fail(ITPP_ERR_ARG, "null argument");
  itpp_status s = check_config(cfg);
  if (s != ITPP_OK) return s;
  int dev = 0;
  hipDeviceProp_t prop;
  s = device_props(&dev, &prop);
  if (s != ITPP_OK) return s;
  return create_impl(cfg, dev, prop, nullptr, 0, nullptr, out);
}

itpp_status itpp_destroy(itpp_ctx ctx) {
  if (!ctx) return ITPP_OK;
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->gate_stream) (void)hipStreamSynchronize(ctx->gate_stream);
  drop_step_graph(ctx);
  if (ctx->gate_stream) (void)hipStreamDestroy(ctx->gate_stream);
  if (ctx->join_in) (void)hipEventDestroy(ctx->join_in);
  if (ctx->join_out) (void)hipEventDestroy(ctx->join_out);
  free_ckpts(ctx);
  free_all(ctx);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->own_stream);
  delete ctx;
  return ITPP_OK;
}

itpp_status itpp_set_hamiltonian(itpp_ctx c, int32_t n_terms, const uint64_t* x, const uint64_t* z,
                                 const double* alpha) {
  if (!c) return ITPP_ERR_ARG;
  if (n_terms < 1 || !x || !z || !alpha) return fail(c, ITPP_ERR_ARG, "empty Hamiltonian");
  const int W = c->W, n = c->n;
  std::vector<TermInfo> terms(n_terms);
  for (int k = 0; k < n_terms; ++k) {
    TermInfo& t = terms[k];
    t.x.assign(x + (size_t)k * W, x + (size_t)k * W + W);
    t.z.assign(z + (size_t)k * W, z + (size_t)k * W + W);
    for (int q = 0; q < W; ++q) {
      const int hi = n - 64 * q;
      if (hi < 64) {
        const uint64_t bad = hi <= 0 ? ~0ull : ~((1ull << hi) - 1ull);
        if ((t.x[q] | t.z[q]) & bad) return fail(c, ITPP_ERR_ARG, "term has bits at or above n_qubits");
      }
    }
    if (!std::isfinite(alpha[k])) return fail(c, ITPP_ERR_ARG, "non-finite term weight");
    t.alpha = alpha[k];
    const int flips = popcount_words(t.x) + popcount_words(t.z);
    if (flips > kMaxClassBits)
      return fail(c, ITPP_ERR_ARG, "term flips more than two bits (|x| + |z| > 2): not supported");
    t.identity = flips == 0;
    for (int j = 0; j < n; ++j) {
      const int xj = (t.x[j >> 6] >> (j & 63)) & 1, zj = (t.z[j >> 6] >> (j & 63)) & 1;
      if (xj) t.F.push_back(j);
      if (zj) t.F.push_back(n + j);
      if (zj) t.cbits.push_back(j);      // x_P z_Q
      if (xj) t.cbits.push_back(n + j);  // z_P x_Q
      if (xj || zj) {
        t.sup[t.nsup] = j;
        t.qx[t.nsup] = xj;
        t.qz[t.nsup] = zj;
        ++t.nsup;
        if (xj && zj) ++t.aQ;
      }
    }
    std::sort(t.F.begin(), t.F.end());
  }
  c->terms.swap(terms);
  c->sched_term.clear();
  c->sched_mult.clear();
  c->glist.clear();
  c->ready = false;
  drop_step_graph(c);
  return ITPP_OK;
}

itpp_status itpp_set_schedule(itpp_ctx c, int32_t n_gates, const int32_t* term_idx, const double* mult) {
  if (!c) return ITPP_ERR_ARG;
  if (c->terms.empty()) return fail(c, ITPP_ERR_STATE, "set_hamiltonian first");
  if (n_gates < 1 || !term_idx || !mult) return fail(c, ITPP_ERR_ARG, "empty schedule");
  std::vector<int> st(n_gates), gl;
  std::vector<double> sm(n_gates);
  for (int g = 0; g < n_gates; ++g) {
    if (term_idx[g] < 0 || term_idx[g] >= (int)c->terms.size())
      return fail(c, ITPP_ERR_ARG, "schedule term index out of range");
    if (!std::isfinite(mult[g])) return fail(c, ITPP_ERR_ARG, "non-finite schedule multiplier");
    st[g] = term_idx[g];
    sm[g] = mult[g];
    if (!c->terms[st[g]].identity) gl.push_back(g);
  }
  c->sched_term.swap(st);
  c->sched_mult.swap(sm);
  c->glist.swap(gl);
  drop_step_graph(c);
  return do_reset(c);
}

itpp_status itpp_reset(itpp_ctx c) {
  if (!c) return ITPP_ERR_ARG;
  return do_reset(c);
}

itpp_status itpp_import(itpp_ctx c, int64_t m, const uint64_t* x, const uint64_t* z, const double* coef) {
  if (!c) return ITPP_ERR_ARG;
  if (m < 1 || !x || !z || !coef) return fail(c, ITPP_ERR_ARG, "empty state");
  if (c->glist.empty()) return fail(c, ITPP_ERR_STATE, "set_hamiltonian and set_schedule first");
  const int W = c->W, NW = c->NW, n = c->n, nbits = c->nbits;
  const double delta = c->cfg.threshold;
  int64_t ident = -1;
  for (int64_t j = 0; j < m; ++j) {
    uint64_t any = 0;
    for (int q = 0; q < W; ++q) {
      const uint64_t xw = x[(size_t)j * W + q], zw = z[(size_t)j * W + q];
      any |= xw | zw;
      const int hi = n - 64 * q;
      if (hi < 64) {
        const uint64_t bad = hi <= 0 ? ~0ull : ~((1ull << hi) - 1ull);
        if ((xw | zw) & bad) return fail(c, ITPP_ERR_ARG, "string has bits at or above n_qubits");
      }
    }
    if (!std::isfinite(coef[j])) return fail(c, ITPP_ERR_ARG, "non-finite coefficient");
    if (any == 0) {
      if (ident >= 0) return fail(c, ITPP_ERR_ARG, "duplicate string (identity)");
      ident = j;
    }
  }
  if (ident < 0) return fail(c, ITPP_ERR_ARG, "the identity string is missing");
  // the context's precision decides the stored value and the threshold test
  auto stored = [&](int64_t j) { return c->f32 ? (double)(float)coef[j] : coef[j]; };
  const double cI = stored(ident);
  if (!(cI > 0.0) || !(cI > delta)) return fail(c, ITPP_ERR_ARG, "identity coefficient must exceed max(0, threshold)");
  // layout of the state after a reset: rep with the first gate's flip bits on
  // top, one producer class, region e = class under the first gate, sorted
  std::vector<int> pos;
  initial_rep(c, pos);
  const int G = (int)c->glist.size();
  const TermInfo& t0 = c->terms[c->sched_term[c->glist[0]]];
  const TermInfo& t1 = c->terms[c->sched_term[c->glist[1 % G]]];
  const int w0 = (int)t0.F.size();
  std::vector<int64_t> keep;
  keep.reserve((size_t)m);
  for (int64_t j = 0; j < m; ++j)
    if (j == ident || std::fabs(stored(j)) > delta) keep.push_back(j);
  const int64_t N = (int64_t)keep.size();
  if (N > c->cfg.max_terms || (uint64_t)N > c->cap)
    return fail(c, ITPP_ERR_ARG, "more strings above the threshold than max_terms");
  std::vector<uint64_t> rk((size_t)N * NW, 0ull);
  for (int64_t k = 0; k < N; ++k) {
    const int64_t j = keep[k];
    uint64_t* key = &rk[(size_t)k * NW];
    for (int q = 0; q < W; ++q)
      for (int part = 0; part < 2; ++part) {
        uint64_t wv = part == 0 ? x[(size_t)j * W + q] : z[(size_t)j * W + q];
        while (wv) {
          const int b = __builtin_ctzll(wv);
          wv &= wv - 1;
          const int p = pos[part * n + 64 * q + b];
          key[p >> 6] |= 1ull << (p & 63);
        }
      }
  }
  auto key_lt = [&](int64_t a, int64_t b) {
    for (int q = NW - 1; q >= 0; --q) {
      const uint64_t ka = rk[(size_t)a * NW + q], kb = rk[(size_t)b * NW + q];
      if (ka != kb) return ka < kb;
    }
    return false;
  };
  std::vector<int64_t> order((size_t)N);
  for (int64_t k = 0; k < N; ++k) order[k] = k;
  std::sort(order.begin(), order.end(), key_lt);
  auto rbit = [&](int64_t k, int p) { return (int)((rk[(size_t)k * NW + (p >> 6)] >> (p & 63)) & 1ull); };
  Plan pl{};
  pl.wc = 0;
  pl.we = w0;
  // host copies are declared before anything is enqueued and outlive the
  // stream synchronisation below
  std::vector<std::vector<uint64_t>> hk(NW, std::vector<uint64_t>((size_t)N));
  std::vector<double> hc64(c->f32 ? 0 : (size_t)N);
  std::vector<float> hc32(c->f32 ? (size_t)N : 0);
  for (int64_t r = 0; r < N; ++r) {
    const int64_t k = order[r];
    if (r > 0 && !key_lt(order[r - 1], k)) return fail(c, ITPP_ERR_ARG, "duplicate string");
    int e = 0, f = 0;
    for (int b = 0; b < w0; ++b) e |= rbit(k, nbits - w0 + b) << b;
    for (int b = 0; b < (int)t1.F.size(); ++b) f |= rbit(k, pos[t1.F[b]]) << b;
    pl.cnt[0][e] += 1;
    pl.ncnt[e][f] += 1;
    for (int q = 0; q < NW; ++q) hk[q][(size_t)r] = rk[(size_t)k * NW + q];
    const double v = coef[keep[k]];
    if (c->f32)
      hc32[(size_t)r] = (float)v;
    else
      hc64[(size_t)r] = v;
  }
  uint64_t acc = 0;
  for (int e = 0; e < kMaxClasses; ++e) {
    pl.base[0][e] = acc;
    acc += pl.cnt[0][e];
  }
  Filter fl{};
  fl.cI = cI;
  fl.n_written = (uint64_t)N;
  fl.n_survivors = (uint64_t)N;
  // from here on a failure leaves no valid state
  c->ready = false;
  free_ckpts(c);
  HIP_TRY(c, launch_init(c->NW, c->f32, c->side[0], c->plan + 0, c->filt + 0, c->ctl, w0, c->stream));
  for (int q = 0; q < NW; ++q)
    HIP_TRY(c, hipMemcpyAsync(c->side[0].kw[q], hk[q].data(), sizeof(uint64_t) * N, hipMemcpyHostToDevice,
                              c->stream));
  if (c->f32)
    HIP_TRY(c, hipMemcpyAsync(c->side[0].coef, hc32.data(), sizeof(float) * N, hipMemcpyHostToDevice, c->stream));
  else
    HIP_TRY(c, hipMemcpyAsync(c->side[0].coef, hc64.data(), sizeof(double) * N, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->plan + 0, &pl, sizeof(Plan), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->filt + 0, &fl, sizeof(Filter), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->pos.swap(pos);
  c->state_hint = (uint64_t)N;
  c->fwd_gates = 0;
  c->fwd_dtau = 0.0;
  c->fwd_valid = true;
  c->cur = 0;
  c->par = 0;
  c->gpos = 0;
  c->ready = true;
  return ITPP_OK;
}

static itpp_status run_gates(itpp_ctx c, double dtau, int64_t n_gates, itpp_stats* st);

itpp_status itpp_evolve(itpp_ctx c, double dtau, int64_t n_steps, itpp_stats* st) {
  if (!c) return ITPP_ERR_ARG;
  if (c->sched_term.empty()) return fail(c, ITPP_ERR_STATE, "set_schedule first");
  if (!(dtau > 0.0) || !std::isfinite(dtau)) return fail(c, ITPP_ERR_ARG, "dtau must be finite and > 0");
  if (n_steps < 0) return fail(c, ITPP_ERR_ARG, "n_steps must be >= 0");
  return run_gates(c, dtau, n_steps * (int64_t)c->glist.size(), st);
}

itpp_status itpp_evolve_gates(itpp_ctx c, double dtau, int64_t n_gates, itpp_stats* st) {
  if (!c) return ITPP_ERR_ARG;
  if (c->sched_term.empty()) return fail(c, ITPP_ERR_STATE, "set_schedule first");
  if (!(dtau > 0.0) || !std::isfinite(dtau)) return fail(c, ITPP_ERR_ARG, "dtau must be finite and > 0");
  if (n_gates < 0) return fail(c, ITPP_ERR_ARG, "n_gates must be >= 0");
  return run_gates(c, dtau, n_gates, st);
}

// Parameters of gate i of the schedule's gate list for a state in rep `pos`;
// pos1 receives the rep of its output and rp the output rep positions.
static itpp_status build_gate(itpp_ctx c, int i, const std::vector<int>& pos, double dtau, bool spec, int shape,
                              GateParams& gp, std::vector<int>& pos1, RepPos& rp) {
  const int G = (int)c->glist.size();
  const int nbits = c->nbits;
  const int sg = c->glist[i];
  const TermInfo& t = c->terms[c->sched_term[sg]];
  const TermInfo& t1 = c->terms[c->sched_term[c->glist[(i + 1) % G]]];
  const TermInfo& t2 = c->terms[c->sched_term[c->glist[(i + 2) % G]]];
  const double theta = t.alpha * c->sched_mult[sg] * dtau;
  std::memset(&gp, 0, sizeof(gp));
  gp.ch = c->real_time ? std::cos(theta) : std::cosh(theta);
  gp.sh = c->real_time ? std::sin(theta) : std::sinh(theta);
  gp.nbits = nbits;
  gp.w = (int)t.F.size();
  gp.w1 = (int)t1.F.size();
  gp.w2 = (int)t2.F.size();
  for (int b : t.cbits) {
    const int p = pos[b];
    gp.cmask[p >> 6] |= 1ull << (p & 63);
  }
  gp.nsup = t.nsup;
  gp.aQ = t.aQ & 3;
  for (int j = 0; j < t.nsup; ++j) {
    gp.px[j] = pos[t.sup[j]];
    gp.pz[j] = pos[c->n + t.sup[j]];
    gp.qx[j] = t.qx[j];
    gp.qz[j] = t.qz[j];
  }
  for (int k = 0; k < gp.w; ++k)
    if (pos[t.F[k]] != nbits - gp.w + k) return fail(c, ITPP_ERR_DEVICE, "internal error: rep invariant");
  pos1 = pos;
  for (int m = 0; m < gp.w1; ++m) {
    gp.epos[m] = pos[t1.F[m]];
    move_top(pos1, t1.F[m], nbits, &gp.mv[m]);
  }
  gp.ov = 0;
  for (int k = 0; k < gp.w1; ++k)
    if (std::find(t.F.begin(), t.F.end(), t1.F[k]) != t.F.end()) gp.ov |= 1 << k;
  gp.ovf = 0;
  for (int b = 0; b < gp.w2; ++b) {
    gp.fpos[b] = pos1[t2.F[b]];
    gp.fposg[b] = pos[t2.F[b]];
    if (std::find(t.F.begin(), t.F.end(), t2.F[b]) != t.F.end()) gp.ovf |= 1 << b;
  }
  for (int k = 0; k < gp.w; ++k) {
    const int q = pos1[t.F[k]];
    gp.qm1[q >> 6] |= 1ull << (q & 63);
  }
  for (int q = 0; q < kMaxKeyWords; ++q) gp.topm[q] = 0;
  for (int b = nbits - gp.w; b < nbits; ++b) gp.topm[b >> 6] |= 1ull << (b & 63);
  // weight change of the branch Q P over P for every support pattern of P
  gp.wmax = c->max_weight;
  gp.pad_wmax = 0;
  gp.wtab = 0;
  for (uint32_t idx = 0; idx < 16; ++idx) {
    int dw = 0;
    for (int j = 0; j < t.nsup && j < 2; ++j) {
      const int xp = (idx >> (2 * j)) & 1, zp = (idx >> (2 * j + 1)) & 1;
      dw += ((xp ^ t.qx[j]) | (zp ^ t.qz[j])) - (xp | zp);
    }
    gp.wtab |= (uint64_t)(dw + 2) << (3 * idx);
  }
  // packed rep positions and the phase table of the layer kernel
  gp.mvpos = 0;
  for (int m = 0; m < gp.w1; ++m) gp.mvpos |= (uint32_t)gp.mv[m] << (8 * m);
  gp.fgpos = 0;
  for (int b = 0; b < gp.w2; ++b) gp.fgpos |= (uint32_t)gp.fposg[b] << (8 * b);
  for (int m = 0; m < gp.w1; ++m) gp.fgpos |= (uint32_t)gp.epos[m] << (16 + 8 * m);
  gp.q1pos = 0;
  for (int k = 0; k < gp.w; ++k) gp.q1pos |= (uint32_t)pos1[t.F[k]] << (8 * k);
  uint32_t phflip = 0;
  gp.phpos = 0;
  for (int j = 0; j < t.nsup; ++j) {
    gp.phpos |= (uint32_t)gp.px[j] << (16 * j);
    gp.phpos |= (uint32_t)gp.pz[j] << (16 * j + 8);
    if (gp.px[j] >= nbits - gp.w) phflip |= 1u << (2 * j);
    if (gp.pz[j] >= nbits - gp.w) phflip |= 1u << (2 * j + 1);
  }
  // e mod 4 of Q P = i^e R for every pattern of (x, z) bits of P on the
  // support of Q (Pauli algebra, the convention of phase_negative)
  gp.etab = 0;
  bool phase_needed = c->real_time;
  for (uint32_t idx = 0; idx < 16; ++idx) {
    int e = t.aQ, anti = 0;
    bool valid = true;
    for (int j = 0; j < 2; ++j) {
      const int xp = (idx >> (2 * j)) & 1, zp = (idx >> (2 * j + 1)) & 1;
      if (j >= t.nsup) {
        if (xp || zp) valid = false;
        continue;
      }
      const int qx = t.qx[j], qz = t.qz[j];
      const int xr = xp ^ qx, zr = zp ^ qz;
      e += (xp & zp) - (xr & zr) + 2 * (qz & xp);
      anti += (xp & qz) ^ (zp & qx);
    }
    e &= 3;
    gp.etab |= (uint32_t)e << (2 * idx);
    if (valid && !(anti & 1) && e != 0) phase_needed = true;
  }
  const uint32_t nph = phase_needed ? (uint32_t)(2 * t.nsup) : 0u;
  gp.lflags = (uint32_t)gp.ov | ((uint32_t)gp.ovf << 2) | ((uint32_t)gp.w2 << 4) | (nph << 6) | (phflip << 9);
  gp.tile = gate_tile(c->NW, shape);
  gp.delta = c->cfg.threshold;
  gp.cap_elems = c->cap;
  gp.status_cap = c->status_cap;
  gp.spec = spec ? 1 : 0;
  gp.spos = i < kRatioSlots ? i : -1;
  gp.spec_mult = c->spec_mult;
  for (int b = 0; b < nbits; ++b) gp.pos_in[b] = (uint8_t)pos[b];
  std::memset(&rp, 0, sizeof(rp));
  rp.nbits = nbits;
  for (int b = 0; b < nbits; ++b) rp.pos[b] = (uint8_t)pos1[b];
  return ITPP_OK;
}

// Gate kernel shape of the next launches: the option, or the size rule of
// kShapeAuto. With forward checkpoints the automatic choice is shape 1, the
// shape the reverse sweep's recomputation is verified with. The layer kernel
// has no weight cutoff, so such gates run on shape 1.
static int effective_shape(itpp_ctx c) {
  int s = c->shape;
  if (s == kShapeAuto) s = (c->ckpt_every == 0 && c->state_hint <= kAutoShapeMaxStrings) ? 2 : 1;
  return (s == 2 && c->max_weight > 0) ? 1 : s;
}

// Plan and enqueue the next elementary gate of the schedule (asynchronous).
static itpp_status enqueue_gate(itpp_ctx c, double dtau, bool spec) {
  const int G = (int)c->glist.size();
  const int i = c->gpos;
  GateParams gp;
  std::vector<int> pos1;
  RepPos rp;
  const int shape = effective_shape(c);
  itpp_status bs = build_gate(c, i, c->pos, dtau, spec, shape, gp, pos1, rp);
  if (bs != ITPP_OK) return bs;
  const int in = c->cur, out = c->cur ^ 1;
  const int pin = c->par, pout = c->par ^ 1;
  HIP_TRY(c, launch_partition(c->NW, gp, c->side[in], c->plan + pin, c->ctl, c->part, c->status, c->stream));
  hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr;
  if (c->timing) {
    if (c->ev_used + 3 > 3 * 4096) HIP_TRY(c, drain_events(c));
    HIP_TRY(c, next_event(c, &e0));
    HIP_TRY(c, next_event(c, &e1));
    HIP_TRY(c, next_event(c, &e2));
    HIP_TRY(c, hipEventRecord(e0, c->stream));
  }
  if (shape == 2)
    HIP_TRY(c, launch_layer(c->NW, c->f32, c->real_time, gp, c->side[in], c->side[out], c->plan + pin, c->plan + pout,
                            c->filt + pin, c->ctl, c->status, c->part, std::max(1, c->cus / c->grid_div), c->stream));
  else
    HIP_TRY(c, (c->real_time ? launch_gate_rt : launch_gate)(
                   c->NW, c->f32, shape, gp, c->side[in], c->side[out], c->plan + pin, c->plan + pout,
                   c->filt + pin, c->ctl, c->status, c->part,
                   std::max(1, c->cus * gate_wgs_per_cu(shape) / c->grid_div), c->stream));
  if (c->timing) HIP_TRY(c, hipEventRecord(e1, c->stream));
  HIP_TRY(c, launch_select(c->NW, c->f32, c->side[out], c->plan + pout, c->filt + pin, c->filt + pout, c->plan + pin,
                           c->ctl, c->sel, rp, c->cfg.max_terms, c->cfg.cap_policy == ITPP_CAP_FAIL ? 1 : 0,
                           gp.spec, gp.spos, c->cus * 4, c->stream));
  if (c->timing) HIP_TRY(c, hipEventRecord(e2, c->stream));
  c->pos.swap(pos1);
  c->cur = out;
  c->par = pout;
  c->gpos = (i + 1) % G;
  c->serial += 1;
  return ITPP_OK;
}

static void drop_step_graph(itpp_ctx c) {
  if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
  c->step_exec = nullptr;
  c->step_pos.clear();
  c->step_snaps.clear();
  c->step_cur = c->step_par = -1;
}

// Trotter steps in one recorded graph: a step of an odd number of gates
// ends in the other ping-pong slots, two of them in the slots they started.
static int graph_period(int G) { return G % 2 ? 2 : 1; }

// Record the launches of graph_period Trotter steps starting at the current
// host state (gpos == 0) as a graph.  Sets *ok = false (nothing recorded)
// if they do not end in the bit order and slots they start from, so that
// the graph could not be replayed.  The host state is unchanged.
static itpp_status record_step(itpp_ctx c, double dtau, bool* ok) {
  *ok = false;
  const int G = (int)c->glist.size() * graph_period((int)c->glist.size());
  const std::vector<int> pos0 = c->pos;
  const int cur0 = c->cur, par0 = c->par;
  const uint64_t serial0 = c->serial;
  std::vector<HostSnap> snaps;
  HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  itpp_status s = ITPP_OK;
  for (int j = 0; j < G && s == ITPP_OK; ++j) {
    snaps.push_back(HostSnap{c->pos, c->cur, c->par, c->gpos, c->serial - serial0, 0});
    s = enqueue_gate(c, dtau, true);
  }
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(c->stream, &g);
  const bool periodic = c->pos == pos0 && c->cur == cur0 && c->par == par0 && c->gpos == 0;
  if (s != ITPP_OK || ee != hipSuccess || !periodic) {
    if (g) (void)hipGraphDestroy(g);
    c->pos = pos0;
    c->cur = cur0;
    c->par = par0;
    c->gpos = 0;
    c->serial = serial0;
    if (s != ITPP_OK) return s;
    if (ee != hipSuccess) return hip_fail(c, ee, "hipStreamEndCapture");
    return ITPP_OK;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  c->pos = pos0;
  c->serial = serial0;
  if (ie != hipSuccess) return hip_fail(c, ie, "hipGraphInstantiate");
  drop_step_graph(c);
  c->step_exec = ex;
  c->step_pos = pos0;
  c->step_cur = cur0;
  c->step_par = par0;
  c->step_dtau = dtau;
  c->step_shape = effective_shape(c);
  c->step_snaps = std::move(snaps);
  *ok = true;
  return ITPP_OK;
}

static itpp_status run_gates_on(itpp_ctx c, double dtau, int64_t n_gates, itpp_stats* st);

static itpp_status run_gates(itpp_ctx c, double dtau, int64_t n_gates, itpp_stats* st) {
  if (c->stream != nullptr || !c->graphs || c->timing || c->ckpt_every > 0) return run_gates_on(c, dtau, n_gates, st);
  if (!c->gate_stream) {
    HIP_TRY(c, hipStreamCreateWithFlags(&c->gate_stream, hipStreamNonBlocking));
    HIP_TRY(c, hipEventCreateWithFlags(&c->join_in, hipEventDisableTiming));
    HIP_TRY(c, hipEventCreateWithFlags(&c->join_out, hipEventDisableTiming));
  }
  HIP_TRY(c, hipEventRecord(c->join_in, nullptr));
  HIP_TRY(c, hipStreamWaitEvent(c->gate_stream, c->join_in, 0));
  c->stream = c->gate_stream;
  const itpp_status s = run_gates_on(c, dtau, n_gates, st);
  c->stream = nullptr;
  HIP_TRY(c, hipEventRecord(c->join_out, c->gate_stream));
  HIP_TRY(c, hipStreamWaitEvent(nullptr, c->join_out, 0));
  return s;
}

static itpp_status run_gates_on(itpp_ctx c, double dtau, int64_t n_gates, itpp_stats* st) {
  if (!c->ready) {
    itpp_status s = do_reset(c);
    if (s != ITPP_OK) return s;
  }
  Ctl h0{};
  HIP_TRY(c, hipMemcpyAsync(&h0, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (h0.error) return check_error(c);
  const double tu0 = h0.term_updates;
  const double ae0 = h0.alg_elems;
  const double we0 = h0.written_elems;
  {
    // restart the run's min / max statistics (three adjacent doubles)
    static const double init[3] = {HUGE_VAL, 0.0, HUGE_VAL};
    static_assert(offsetof(Ctl, cI_max) == offsetof(Ctl, cI_min) + 8 && offsetof(Ctl, kth_min) == offsetof(Ctl, cI_min) + 16,
                  "adjacent statistics");
    HIP_TRY(c, hipMemcpyAsync(&c->ctl->cI_min, init, sizeof(init), hipMemcpyHostToDevice, c->stream));
  }
  const uint64_t g0 = h0.gates;
  const uint64_t sg0 = h0.spec_gates;
  c->serial = h0.gate_serial;
  const int G = (int)c->glist.size();
  int64_t retries = 0;
  int64_t done = 0;
  bool nospec_next = false;
  std::vector<HostSnap> snaps;
  if (n_gates > 0 && G > 0 && c->real_time) {
    c->fwd_valid = false;  // the reverse sweep replays imaginary-time gates only
    free_ckpts(c);
  }
  if (n_gates > 0 && G > 0) {
    if (c->fwd_gates == 0) {
      c->fwd_dtau = dtau;
    } else if (dtau != c->fwd_dtau) {
      c->fwd_valid = false;  // the reverse sweep assumes one dtau since reset
      free_ckpts(c);
    }
  }
  const int64_t E = (int64_t)c->ckpt_every * G;
  // Gates are enqueued in batches; after each batch the host checks whether
  // a speculative gate asked to be redone (all kernels after it were no-ops,
  // so that gate's input is intact) and replays from there without
  // speculation for that gate.
  const bool can_graph = c->graphs && E == 0 && !c->timing && c->stream != nullptr && c->speculate && G > 0;
  const int GR = G * graph_period(G);  // gates in one recorded graph
  const int64_t g_steps0 = c->graph_steps;
  while (done < n_gates && G > 0) {
    // with step graphs, batches end on step boundaries
    const int64_t span = can_graph ? (G - c->gpos) % G + std::max<int64_t>(1, kSyncEvery / GR) * GR : kSyncEvery;
    int64_t batch = std::min<int64_t>(n_gates - done, span);
    if (c->short_batches > 0) {
      // with step graphs a short batch still holds one whole recorded step
      const int64_t lim = can_graph ? (G - c->gpos) % G + GR : kSyncAfterHalt;
      batch = std::min<int64_t>(batch, lim);
      --c->short_batches;
    }
    if (E > 0 && c->fwd_valid) {
      // forward checkpoint of the state before gate fwd_gates, every E gates
      if (c->fwd_gates % E == 0 && (int64_t)c->ckpts.size() == c->fwd_gates / E) {
        uint64_t cnt = 0;
        HIP_TRY(c, state_count(c, &cnt));
        void* mem = nullptr;
        if (hipMalloc(&mem, snapshot_bytes(c, cnt)) != hipSuccess) {
          (void)hipGetLastError();
          return fail(c, ITPP_ERR_OOM, "no device memory for a forward checkpoint");
        }
        Snapshot sn;
        sn.owned = mem;
        hipError_t he = write_snapshot(c, sn, mem, cnt);
        c->ckpts.push_back(sn);
        if (he != hipSuccess) return hip_fail(c, he, "forward checkpoint");
      }
      batch = std::min<int64_t>(batch, E - c->fwd_gates % E);
    }
    snaps.clear();
    // whole Trotter steps run as replays of a recorded graph when they can
    // (no checkpoints or event timing, a stream that can be captured and a
    // speculative first gate)
    for (int64_t b = 0; b < batch;) {
      if (c->gpos == 0 && can_graph && !(b == 0 && nospec_next) && batch - b >= GR) {
        bool have = c->step_exec && c->step_pos == c->pos && c->step_cur == c->cur && c->step_par == c->par &&
                    c->step_dtau == dtau && c->step_shape == effective_shape(c);
        // record once the step-start bit order repeats (from the second step)
        if (!have && c->last_step_pos == c->pos) {
          itpp_status s = record_step(c, dtau, &have);
          if (s != ITPP_OK) return s;
        }
        c->last_step_pos = c->pos;
        if (have) {
          for (int j = 0; j < GR; ++j) {
            HostSnap sn = c->step_snaps[j];
            sn.serial += c->serial;
            snaps.push_back(std::move(sn));
          }
          HIP_TRY(c, hipGraphLaunch(c->step_exec, c->stream));
          c->serial += (uint64_t)GR;
          c->graph_steps += graph_period(G);
          b += GR;
          continue;
        }
      } else if (c->gpos == 0) {
        c->last_step_pos = c->pos;
      }
      snaps.push_back(HostSnap{c->pos, c->cur, c->par, c->gpos, c->serial, c->ev_used});
      // with checkpoints the forward writes exactly what a recomputation
      // writes (no speculation), so stored states pack to the same layout
      const bool spec = c->speculate && E == 0 && !(b == 0 && nospec_next);
      itpp_status s = enqueue_gate(c, dtau, spec);
      if (s != ITPP_OK) return s;
      ++b;
    }
    nospec_next = false;
    Ctl h{};
    Filter fl{};
    HIP_TRY(c, hipMemcpyAsync(&h, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    // the state's size, for the automatic gate kernel shape of the next batch
    if (c->shape == kShapeAuto)
      HIP_TRY(c, hipMemcpyAsync(&fl, c->filt + c->par, sizeof(Filter), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (h.error) return check_error(c);
    if (h.halt) {
      const int64_t idx = (int64_t)(h.halt_serial - snaps[0].serial);
      if (idx < 0 || idx >= batch) return fail(c, ITPP_ERR_DEVICE, "internal error: bad retry serial");
      const HostSnap& sn = snaps[idx];
      c->pos = sn.pos;
      c->cur = sn.cur;
      c->par = sn.par;
      c->gpos = sn.gpos;
      c->serial = h.halt_serial + 1;  // the redone gate's serial on the device
      // keep the timing of the failed attempt, drop the no-op launches after it
      if (c->timing) c->ev_used = std::min(c->ev_used, sn.ev_used + 3);
      HIP_TRY(c, launch_prepare(c->plan + (c->par ^ 1), c->ctl, c->stream));
      done += idx;
      c->fwd_gates += idx;
      nospec_next = true;
      ++retries;
      c->short_batches = kShortBatchesAfterHalt;
      continue;
    }
    if (c->shape == kShapeAuto) c->state_hint = fl.n_survivors;
    done += batch;
    c->fwd_gates += batch;
  }
  c->retries_total += retries;
  if (st) {
    Ctl h{};
    Filter f{};
    HIP_TRY(c, hipMemcpyAsync(&h, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(&f, c->filt + c->par, sizeof(Filter), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    st->n_terms = (int64_t)f.n_survivors;
    st->n_gates = (int64_t)(h.gates - g0);
    st->term_updates = h.term_updates - tu0;
    st->c_identity = f.cI;
    st->cap_hit = (int32_t)h.cap_hit;
    st->alg_bytes = (h.alg_elems - ae0) * (double)(8 * c->NW + c->coef_bytes);
    st->spec_gates = (int64_t)(h.spec_gates - sg0);
    st->spec_retries = retries;
    st->written = h.written_elems - we0;
    st->c_I_min = h.cI_min;
    st->c_I_max = h.cI_max;
    st->kth_abs_min = h.kth_min;
    st->graph_steps = c->graph_steps - g_steps0;
  }
  if (c->timing) {
    Ctl h{};
    HIP_TRY(c, hipMemcpyAsync(&h, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->t_alg_bytes += (h.alg_elems - ae0) * (double)(8 * c->NW + c->coef_bytes);
  }
  return ITPP_OK;
}

itpp_status itpp_set_option(itpp_ctx c, int32_t option, double value) {
  if (!c) return ITPP_ERR_ARG;
  // a recorded step holds the launch arguments of the old settings
  drop_step_graph(c);
  switch (option) {
    case ITPP_OPT_SPECULATION:
      if (value != 0.0 && value != 1.0) return fail(c, ITPP_ERR_ARG, "speculation must be 0 or 1");
      c->speculate = value != 0.0;
      return ITPP_OK;
    case ITPP_OPT_SPEC_MARGIN:
      if (!(value > 0.0) || !(value <= 1.0)) return fail(c, ITPP_ERR_ARG, "margin must be in (0, 1]");
      c->spec_mult = value;
      return ITPP_OK;
    case ITPP_OPT_GATE_SHAPE:
      if (value != 0.0 && value != 1.0 && value != 2.0 && value != (double)kShapeAuto)
        return fail(c, ITPP_ERR_ARG, "gate shape must be 0, 1, 2 or 3 (automatic)");
      c->shape = (int)value;
      return ITPP_OK;
    case ITPP_OPT_REAL_TIME:
      if (value != 0.0 && value != 1.0) return fail(c, ITPP_ERR_ARG, "real time must be 0 or 1");
      c->real_time = value != 0.0;
      // the reverse sweep replays imaginary-time gates only
      if (c->real_time) {
        c->fwd_valid = false;
        free_ckpts(c);
      }
      return ITPP_OK;
    case ITPP_OPT_GRAPHS:
      if (value != 0.0 && value != 1.0) return fail(c, ITPP_ERR_ARG, "graphs must be 0 or 1");
      c->graphs = value != 0.0;
      return ITPP_OK;
    case ITPP_OPT_MAX_WEIGHT:
      if (!(value >= 0.0) || value > (double)c->n || value != std::floor(value))
        return fail(c, ITPP_ERR_ARG, "weight cutoff must be an integer in [0, n]");
      if (value > 0.0 && c->ckpt_every > 0) return fail(c, ITPP_ERR_STATE, "the reverse sweep has no weight cutoff");
      c->max_weight = (int)value;
      return ITPP_OK;
    case ITPP_OPT_GRID_DIV:
      if (value != 1.0 && value != 2.0 && value != 4.0 && value != 8.0)
        return fail(c, ITPP_ERR_ARG, "grid divisor must be 1, 2, 4 or 8");
      c->grid_div = (int)value;
      return ITPP_OK;
    default:
      return fail(c, ITPP_ERR_ARG, "unknown option");
  }
}

itpp_status itpp_set_timing(itpp_ctx c, int32_t enable) {
  if (!c) return ITPP_ERR_ARG;
  HIP_TRY(c, drain_events(c));
  c->timing = enable != 0;
  c->t_gate_ms = c->t_sel_ms = c->t_alg_bytes = 0.0;
  c->t_gates = 0;
  return ITPP_OK;
}

itpp_status itpp_get_timing(itpp_ctx c, itpp_timing* out) {
  if (!c || !out) return ITPP_ERR_ARG;
  HIP_TRY(c, drain_events(c));
  out->gate_ms = c->t_gate_ms;
  out->select_ms = c->t_sel_ms;
  out->gate_launches = c->t_gates;
  out->alg_bytes = c->t_alg_bytes;
  return ITPP_OK;
}

itpp_status itpp_num_terms(itpp_ctx c, int64_t* out) {
  if (!c || !out) return ITPP_ERR_ARG;
  if (!c->ready) return fail(c, ITPP_ERR_STATE, "no valid state (reset required)");
  Filter f{};
  HIP_TRY(c, hipMemcpyAsync(&f, c->filt + c->par, sizeof(Filter), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *out = (int64_t)f.n_survivors;
  return ITPP_OK;
}

itpp_status itpp_expect(itpp_ctx c, int32_t m, const uint64_t* x, const uint64_t* z, const double* coef,
                        double* out) {
  if (!c || !out) return ITPP_ERR_ARG;
  if (m < 0 || (m > 0 && (!x || !z || !coef))) return fail(c, ITPP_ERR_ARG, "bad observable arrays");
  if (!c->ready) return fail(c, ITPP_ERR_STATE, "no valid state (reset required)");
  const int W = c->W;
  for (int j = 0; j < m; ++j)
    for (int q = 0; q < W; ++q) {
      const int hi = c->n - 64 * q;
      if (hi < 64) {
        const uint64_t bad = hi <= 0 ? ~0ull : ~((1ull << hi) - 1ull);
        if ((x[(size_t)j * W + q] | z[(size_t)j * W + q]) & bad)
          return fail(c, ITPP_ERR_ARG, "observable has bits at or above n_qubits");
      }
    }
  if (m == 0) {
    *out = 0.0;
    return ITPP_OK;
  }
  double r = 0.0;  // outlives the device buffers, whose release waits for the copy into it
  DevBuf bx, bz, bc;
  HIP_TRY(c, bx.alloc(sizeof(uint64_t) * m * W));
  HIP_TRY(c, bz.alloc(sizeof(uint64_t) * m * W));
  HIP_TRY(c, bc.alloc(sizeof(double) * m));
  HIP_TRY(c, hipMemcpyAsync(bx.p, x, sizeof(uint64_t) * m * W, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(bz.p, z, sizeof(uint64_t) * m * W, hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(bc.p, coef, sizeof(double) * m, hipMemcpyHostToDevice, c->stream));
  RepPos rp{};
  rp.nbits = c->nbits;
  for (int b = 0; b < c->nbits; ++b) rp.pos[b] = (uint8_t)c->pos[b];
  HIP_TRY(c, launch_observe(c->NW, c->f32, c->side[c->cur], c->plan + c->par, c->filt + c->par, rp,
                            bx.as<uint64_t>(), bz.as<uint64_t>(), bc.as<double>(), m, c->d_result, c->ctl,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(&r, c->d_result, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *out = r;
  return ITPP_OK;
}

itpp_status itpp_export(itpp_ctx c, int64_t capacity, uint64_t* x, uint64_t* z, double* coef, int64_t* n_out) {
  if (!c || !n_out) return ITPP_ERR_ARG;
  if (!c->ready) return fail(c, ITPP_ERR_STATE, "no valid state (reset required)");
  int64_t nt = 0;
  itpp_status s = itpp_num_terms(c, &nt);
  if (s != ITPP_OK) return s;
  if (capacity < nt || !x || !z || !coef) {
    *n_out = nt;
    return fail(c, ITPP_ERR_ARG, "export capacity too small");
  }
  const int W = c->W;
  // host buffers first: they must outlive the device buffers, whose release
  // waits for copies still in flight into them
  unsigned long long cnt = 0;
  std::vector<uint64_t> hx((size_t)nt * W), hz((size_t)nt * W);
  std::vector<double> hc(nt);
  DevBuf bx, bz, bc, bn;
  HIP_TRY(c, bx.alloc(sizeof(uint64_t) * std::max<int64_t>(nt, 1) * W));
  HIP_TRY(c, bz.alloc(sizeof(uint64_t) * std::max<int64_t>(nt, 1) * W));
  HIP_TRY(c, bc.alloc(sizeof(double) * std::max<int64_t>(nt, 1)));
  HIP_TRY(c, bn.alloc(sizeof(unsigned long long)));
  HIP_TRY(c, hipMemsetAsync(bn.p, 0, sizeof(unsigned long long), c->stream));
  RepPos rp{};
  rp.nbits = c->nbits;
  for (int b = 0; b < c->nbits; ++b) rp.pos[b] = (uint8_t)c->pos[b];
  HIP_TRY(c, launch_export(c->NW, c->f32, c->side[c->cur], c->plan + c->par, c->filt + c->par, rp,
                           bx.as<uint64_t>(), bz.as<uint64_t>(), bc.as<double>(), bn.as<unsigned long long>(),
                           (uint64_t)nt, c->cus * 4, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&cnt, bn.p, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
  if (nt > 0) {
    HIP_TRY(c, hipMemcpyAsync(hx.data(), bx.p, sizeof(uint64_t) * nt * W, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(hz.data(), bz.p, sizeof(uint64_t) * nt * W, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(hc.data(), bc.p, sizeof(double) * nt, hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if ((int64_t)cnt != nt) return fail(c, ITPP_ERR_DEVICE, "internal error: export count mismatch");
  std::vector<int64_t> order(nt);
  for (int64_t i = 0; i < nt; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    for (int q = W - 1; q >= 0; --q)
      if (hx[a * W + q] != hx[b * W + q]) return hx[a * W + q] < hx[b * W + q];
    for (int q = W - 1; q >= 0; --q)
      if (hz[a * W + q] != hz[b * W + q]) return hz[a * W + q] < hz[b * W + q];
    return false;
  });
  for (int64_t i = 0; i < nt; ++i) {
    for (int q = 0; q < W; ++q) {
      x[i * W + q] = hx[order[i] * W + q];
      z[i * W + q] = hz[order[i] * W + q];
    }
    coef[i] = hc[order[i]];
  }
  *n_out = nt;
  return ITPP_OK;
}

itpp_status itpp_expect_squared(itpp_ctx c, int32_t m, const uint64_t* x, const uint64_t* z, const double* coef,
                                double* value, double* purity) {
  if (!c || !value || !purity) return ITPP_ERR_ARG;
  if (m < 0 || (m > 0 && (!x || !z || !coef))) return fail(c, ITPP_ERR_ARG, "bad observable arrays");
  if (!c->ready) return fail(c, ITPP_ERR_STATE, "no valid state (reset required)");
  const int W = c->W, NW = c->NW, n = c->n;
  std::vector<uint64_t> qmask((size_t)std::max(m, 1) * NW, 0ull), cmask((size_t)std::max(m, 1) * NW, 0ull);
  std::vector<int32_t> sup_off(m + 1, 0), sup_pos, sup_q, aq(std::max(m, 1), 0);
  std::vector<double> oc(std::max(m, 1), 0.0);
  auto set_rep = [&](std::vector<uint64_t>& v, int j, int cb) {
    const int p = c->pos[cb];
    v[(size_t)j * NW + (p >> 6)] |= 1ull << (p & 63);
  };
  for (int j = 0; j < m; ++j) {
    if (!std::isfinite(coef[j])) return fail(c, ITPP_ERR_ARG, "non-finite observable weight");
    for (int q = 0; q < W; ++q) {
      const int hi = n - 64 * q;
      if (hi < 64) {
        const uint64_t bad = hi <= 0 ? ~0ull : ~((1ull << hi) - 1ull);
        if ((x[(size_t)j * W + q] | z[(size_t)j * W + q]) & bad)
          return fail(c, ITPP_ERR_ARG, "observable has bits at or above n_qubits");
      }
    }
    for (int i = 0; i < n; ++i) {
      const int xi = (int)((x[(size_t)j * W + (i >> 6)] >> (i & 63)) & 1ull);
      const int zi = (int)((z[(size_t)j * W + (i >> 6)] >> (i & 63)) & 1ull);
      if (!xi && !zi) continue;
      if (xi) {
        set_rep(qmask, j, i);
        set_rep(cmask, j, n + i);  // x_Q z_P
      }
      if (zi) {
        set_rep(qmask, j, n + i);
        set_rep(cmask, j, i);  // z_Q x_P
      }
      sup_pos.push_back(c->pos[i]);
      sup_pos.push_back(c->pos[n + i]);
      sup_q.push_back(xi | (zi << 1));
      aq[j] += xi & zi;
    }
    aq[j] &= 3;
    sup_off[j + 1] = (int32_t)sup_q.size();
    oc[j] = coef[j];
  }
  if (sup_q.empty()) {
    sup_q.push_back(0);
    sup_pos.assign(2, 0);
  }
  const int grid = c->cus * 4;
  double res[2] = {0.0, 0.0};  // outlives the device buffers, whose release waits for the copy into it
  DevBuf bq, bc, boff, bpos, bql, baq, bco, bpart, bout;
  HIP_TRY(c, bq.alloc(sizeof(uint64_t) * qmask.size()));
  HIP_TRY(c, bc.alloc(sizeof(uint64_t) * cmask.size()));
  HIP_TRY(c, boff.alloc(sizeof(int32_t) * sup_off.size()));
  HIP_TRY(c, bpos.alloc(sizeof(int32_t) * sup_pos.size()));
  HIP_TRY(c, bql.alloc(sizeof(int32_t) * sup_q.size()));
  HIP_TRY(c, baq.alloc(sizeof(int32_t) * aq.size()));
  HIP_TRY(c, bco.alloc(sizeof(double) * oc.size()));
  HIP_TRY(c, bpart.alloc(sizeof(double) * 4 * (size_t)grid));
  HIP_TRY(c, bout.alloc(sizeof(double) * 2));
  HIP_TRY(c, hipMemcpyAsync(bq.p, qmask.data(), sizeof(uint64_t) * qmask.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(bc.p, cmask.data(), sizeof(uint64_t) * cmask.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(boff.p, sup_off.data(), sizeof(int32_t) * sup_off.size(), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(bpos.p, sup_pos.data(), sizeof(int32_t) * sup_pos.size(), hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(bql.p, sup_q.data(), sizeof(int32_t) * sup_q.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(baq.p, aq.data(), sizeof(int32_t) * aq.size(), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemcpyAsync(bco.p, oc.data(), sizeof(double) * oc.size(), hipMemcpyHostToDevice, c->stream));
  SqObs ob{};
  ob.m = m;
  ob.qmask = bq.as<uint64_t>();
  ob.cmask = bc.as<uint64_t>();
  ob.sup_off = boff.as<int32_t>();
  ob.sup_pos = bpos.as<int32_t>();
  ob.sup_q = bql.as<int32_t>();
  ob.aq = baq.as<int32_t>();
  ob.coef = bco.as<double>();
  RepPos rp{};
  rp.nbits = c->nbits;
  for (int b = 0; b < c->nbits; ++b) rp.pos[b] = (uint8_t)c->pos[b];
  HIP_TRY(c, launch_squared(c->NW, c->f32, c->side[c->cur], c->plan + c->par, c->filt + c->par, rp, ob, c->ctl,
                            bpart.as<double>(), bout.as<double>(), grid, c->stream));
  HIP_TRY(c, hipMemcpyAsync(res, bout.p, sizeof(res), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  itpp_status st = check_error(c);
  if (st != ITPP_OK) return st;
  *purity = res[1];
  *value = res[0] / res[1];
  return ITPP_OK;
}

itpp_status itpp_expect_squared_noalloc(itpp_ctx c, int32_t m, const uint64_t* x, const uint64_t* z,
                                       const double* coef, double* value, double* purity) {
  if (!c || !value || !purity) return ITPP_ERR_ARG;
  if (m < 0 || (m > 0 && (!x || !z || !coef))) return fail(c, ITPP_ERR_ARG, "bad observable arrays");
  if (m > kSqMaxStrings) return fail(c, ITPP_ERR_ARG, "more than 4096 observable strings (the scratch limit)");
  if (!c->ready) return fail(c, ITPP_ERR_STATE, "no valid state (reset required)");
  const int W = c->W, n = c->n;
  int64_t support = 0;
  for (int j = 0; j < m; ++j) {
    if (!std::isfinite(coef[j])) return fail(c, ITPP_ERR_ARG, "non-finite observable weight");
    for (int q = 0; q < W; ++q) {
      const uint64_t xw = x[(size_t)j * W + q], zw = z[(size_t)j * W + q];
      const int hi = n - 64 * q;
      if (hi < 64) {
        const uint64_t bad = hi <= 0 ? ~0ull : ~((1ull << hi) - 1ull);
        if ((xw | zw) & bad) return fail(c, ITPP_ERR_ARG, "observable has bits at or above n_qubits");
      }
      support += __builtin_popcountll(xw | zw);
    }
  }
  if (support > kSqMaxSupport)
    return fail(c, ITPP_ERR_ARG, "observable strings have more than 65536 non-identity sites in total (the scratch limit)");
  void* sp = nullptr;
  {
    const hipError_t e = scratch_address(c->device, &sp);
    if (e != hipSuccess) return hip_fail(c, e, "scratch address");
  }
  uint8_t* base = static_cast<uint8_t*>(sp);
  const int grid = std::min(c->cus * 4, kSqMaxGrid);
  uint64_t* dx = reinterpret_cast<uint64_t*>(base + kSqOffX);
  uint64_t* dz = reinterpret_cast<uint64_t*>(base + kSqOffZ);
  double* doc = reinterpret_cast<double*>(base + kSqOffOc);
  SqTables t{};
  t.qmask = reinterpret_cast<uint64_t*>(base + kSqOffQ);
  t.cmask = reinterpret_cast<uint64_t*>(base + kSqOffC);
  t.sup_off = reinterpret_cast<int32_t*>(base + kSqOffSupOff);
  t.sup_pos = reinterpret_cast<int32_t*>(base + kSqOffSupPos);
  t.sup_q = reinterpret_cast<int32_t*>(base + kSqOffSupQ);
  t.aq = reinterpret_cast<int32_t*>(base + kSqOffAq);
  t.coef = reinterpret_cast<double*>(base + kSqOffCoef);
  double* part = reinterpret_cast<double*>(base + kSqOffPart);
  double* out = reinterpret_cast<double*>(base + kSqOffOut);
  RepPos rp{};
  rp.nbits = c->nbits;
  for (int b = 0; b < c->nbits; ++b) rp.pos[b] = (uint8_t)c->pos[b];
  if (m > 0) {
    HIP_TRY(c, hipMemcpyAsync(dx, x, sizeof(uint64_t) * m * W, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(dz, z, sizeof(uint64_t) * m * W, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(doc, coef, sizeof(double) * m, hipMemcpyHostToDevice, c->stream));
  }
  HIP_TRY(c, launch_sq_tables(rp, n, W, c->NW, dx, dz, doc, m, t, c->stream));
  SqObs ob{};
  ob.m = m;
  ob.qmask = t.qmask;
  ob.cmask = t.cmask;
  ob.sup_off = t.sup_off;
  ob.sup_pos = t.sup_pos;
  ob.sup_q = t.sup_q;
  ob.aq = t.aq;
  ob.coef = t.coef;
  HIP_TRY(c, launch_squared(c->NW, c->f32, c->side[c->cur], c->plan + c->par, c->filt + c->par, rp, ob, c->ctl, part,
                            out, grid, c->stream));
  double res[2] = {0.0, 0.0};
  HIP_TRY(c, hipMemcpyAsync(res, out, sizeof(res), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  itpp_status st = check_error(c);
  if (st != ITPP_OK) return st;
  *purity = res[1];
  *value = res[0] / res[1];
  return ITPP_OK;
}

itpp_status itpp_expect_device(itpp_ctx c, int32_t m, const uint64_t* x, const uint64_t* z, const double* coef,
                               double* out) {
  if (!c || !out) return ITPP_ERR_ARG;
  if (m < 0 || (m > 0 && (!x || !z || !coef))) return fail(c, ITPP_ERR_ARG, "bad observable arrays");
  if (!c->ready) return fail(c, ITPP_ERR_STATE, "no valid state (reset required)");
  RepPos rp{};
  rp.nbits = c->nbits;
  for (int b = 0; b < c->nbits; ++b) rp.pos[b] = (uint8_t)c->pos[b];
  HIP_TRY(c, launch_observe(c->NW, c->f32, c->side[c->cur], c->plan + c->par, c->filt + c->par, rp, x, z, coef, m,
                            out, c->ctl, c->stream));
  return ITPP_OK;
}

itpp_status itpp_export_device(itpp_ctx c, int64_t capacity, uint64_t* x, uint64_t* z, double* coef,
                               int64_t* n_out) {
  if (!c || !n_out) return ITPP_ERR_ARG;
  if (!c->ready) return fail(c, ITPP_ERR_STATE, "no valid state (reset required)");
  int64_t nt = 0;
  itpp_status s = itpp_num_terms(c, &nt);
  if (s != ITPP_OK) return s;
  if (capacity < nt || !x || !z || !coef) {
    *n_out = nt;
    return fail(c, ITPP_ERR_ARG, "export capacity too small");
  }
  RepPos rp{};
  rp.nbits = c->nbits;
  for (int b = 0; b < c->nbits; ++b) rp.pos[b] = (uint8_t)c->pos[b];
  unsigned long long cnt = 0;
  HIP_TRY(c, hipMemsetAsync(c->d_count, 0, sizeof(unsigned long long), c->stream));
  HIP_TRY(c, launch_export(c->NW, c->f32, c->side[c->cur], c->plan + c->par, c->filt + c->par, rp, x, z, coef,
                           c->d_count, (uint64_t)nt, c->cus * 4, c->stream));
  HIP_TRY(c, hipMemcpyAsync(&cnt, c->d_count, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if ((int64_t)cnt != nt) return fail(c, ITPP_ERR_DEVICE, "internal error: export count mismatch");
  *n_out = nt;
  return ITPP_OK;
}

}  // extern "C"

namespace {

struct Arena {
  uint8_t* base = nullptr;
  uint64_t size = 0, top = 0;
  void* take(uint64_t b) {
    b = (b + 255) & ~255ull;
    if (top + b > size) return nullptr;
    void* p = base + top;
    top += b;
    return p;
  }
};

// Snapshot of the stored state taken from the arena.
itpp_status snap_in_arena(itpp_ctx c, Arena& ar, Snapshot& s) {
  uint64_t cnt = 0;
  HIP_TRY(c, state_count(c, &cnt));
  void* mem = ar.take(snapshot_bytes(c, cnt));
  if (!mem)
    return fail(c, ITPP_ERR_OOM,
                "reverse-sweep workspace too small: raise it or checkpoint more often (itpp_set_adjoint)");
  HIP_TRY(c, write_snapshot(c, s, mem, cnt));
  return ITPP_OK;
}

// Recompute one gate without speculation (the layout the reverse sweep replays).
itpp_status replay_gate(itpp_ctx c) {
  itpp_status st = enqueue_gate(c, c->fwd_dtau, false);
  if (st != ITPP_OK) return st;
  ++c->fwd_gates;
  return ITPP_OK;
}

struct AdjBuffers {
  double* lam[2];
  double* sdev;     // [2]
  double* part;     // 4 per tile
  uint64_t* ntiles;
  double* dtheta;   // per gate since reset
};

// Reverse step of gate g from its input snapshot Sin and output snapshot Sout.
itpp_status adjoint_gate(itpp_ctx c, int64_t g, const Snapshot& Sin, const Snapshot& Sout, AdjBuffers& B, int cur) {
  const int G = (int)c->glist.size();
  const int i = (int)(g % G);
  if (Sin.gpos != i) return fail(c, ITPP_ERR_DEVICE, "internal error: snapshot out of step");
  GateParams gp;
  std::vector<int> pos1;
  RepPos rp;
  itpp_status bs = build_gate(c, i, Sin.pos, c->fwd_dtau, false, 0, gp, pos1, rp);
  if (bs != ITPP_OK) return bs;
  HIP_TRY(c, launch_partition(c->NW, gp, Sin.side, Sin.plan, c->ctl, c->part, c->status, c->stream));
  AdjArgs a{};
  a.lam_out = B.lam[cur];
  a.lam_in = B.lam[cur ^ 1];
  a.plan_next = Sout.plan;
  a.filt_next = Sout.filt;
  a.s_in = B.sdev + cur;
  a.part = B.part;
  a.ntiles = B.ntiles;
  a.lam_out_len = Sout.count;
  HIP_TRY(c, launch_adjoint_gate(c->NW, gp, Sin.side, Sin.plan, c->plan + (c->par ^ 1), Sin.filt, c->ctl, c->status,
                                 c->part, a, c->cus * gate_wgs_per_cu(0), c->stream));
  HIP_TRY(c, launch_adj_reduce(B.part, B.ntiles, B.dtheta + g, B.sdev + (cur ^ 1), c->ctl, c->stream));
  return ITPP_OK;
}

// Compensated sum (Neumaier) on the host.
struct HostSum {
  double s = 0.0, c = 0.0;
  void add(double v) {
    const double t = s + v;
    if (std::fabs(s) >= std::fabs(v))
      c += (s - t) + v;
    else
      c += (v - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

itpp_status backward_impl(itpp_ctx c, int32_t m, const uint64_t* dx, const uint64_t* dz, const double* dc,
                          double* value, double* d_alpha, double* d_dtau, double* d_theta, Arena& ar,
                          AdjBuffers& B) {
  const int64_t Gtot = c->fwd_gates;
  const int nck = (int)c->ckpts.size();
  // the final state: packed copy (restored at the end), L and the seed lambda
  Snapshot SF;
  itpp_status st = snap_in_arena(c, ar, SF);
  if (st != ITPP_OK) return st;
  RepPos rpF{};
  rpF.nbits = c->nbits;
  for (int b = 0; b < c->nbits; ++b) rpF.pos[b] = (uint8_t)SF.pos[b];
  HIP_TRY(c, launch_observe(c->NW, c->f32, SF.side, SF.plan, SF.filt, rpF, dx, dz, dc, m, B.sdev, c->ctl, c->stream));
  HIP_TRY(c, hipMemsetAsync(B.lam[0], 0, std::max<uint64_t>(SF.count, 1) * sizeof(double), c->stream));
  if (m > 0) HIP_TRY(c, launch_seed(c->NW, SF.side, SF.plan, SF.filt, rpF, dx, dz, dc, m, B.lam[0], c->stream));
  HIP_TRY(c, hipMemcpyAsync(value, B.sdev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  int cur = 0;
  const uint64_t keep_top = ar.top;
  for (int k = nck - 1; k >= 0; --k) {
    const int64_t a = c->ckpts[k].gate;
    const int64_t b = (k + 1 < nck) ? c->ckpts[k + 1].gate : Gtot;
    if (b <= a) continue;
    const int64_t L = b - a;
    ar.top = keep_top;
    // Every state of the segment fits in the workspace (a stored state holds
    // at most two outputs per survivor, 2K + 1 strings): one block, recomputed
    // once.  Otherwise blocks of about sqrt(L) gates from sub-checkpoints of a
    // first recomputation, so the segment is recomputed twice.
    const uint64_t snap_max = snapshot_bytes(c, 2 * (uint64_t)c->cfg.max_terms + 64) + 256;
    const bool whole = ar.size - ar.top >= (uint64_t)(L + 1) * snap_max;
    int64_t sblk = whole ? L : (int64_t)std::ceil(std::sqrt((double)L));
    if (sblk < 1) sblk = 1;
    std::vector<Snapshot> subs;
    Snapshot s0 = c->ckpts[k];
    s0.owned = nullptr;
    subs.push_back(s0);
    if (!whole) {
      // sub-checkpoints every sblk gates of the segment
      HIP_TRY(c, restore_snapshot(c, c->ckpts[k]));
      for (int64_t g = a; g < b - 1; ++g) {
        st = replay_gate(c);
        if (st != ITPP_OK) return st;
        if ((c->fwd_gates - a) % sblk == 0) {
          Snapshot sn;
          st = snap_in_arena(c, ar, sn);
          if (st != ITPP_OK) return st;
          subs.push_back(sn);
        }
      }
      st = check_error(c);
      if (st != ITPP_OK) return st;
    }
    const uint64_t sub_top = ar.top;
    const int64_t nblk = (L + sblk - 1) / sblk;
    for (int64_t q = nblk - 1; q >= 0; --q) {
      ar.top = sub_top;
      const int64_t m0 = a + q * sblk, m1 = std::min<int64_t>(b, m0 + sblk);
      HIP_TRY(c, restore_snapshot(c, subs[q]));
      std::vector<Snapshot> sn(m1 - m0 + 1);
      for (int64_t g = m0; g <= m1; ++g) {
        st = snap_in_arena(c, ar, sn[g - m0]);
        if (st != ITPP_OK) return st;
        if (g < m1) {
          st = replay_gate(c);
          if (st != ITPP_OK) return st;
        }
      }
      for (int64_t g = m1 - 1; g >= m0; --g) {
        st = adjoint_gate(c, g, sn[g - m0], sn[g - m0 + 1], B, cur);
        if (st != ITPP_OK) return st;
        cur ^= 1;
      }
      st = check_error(c);
      if (st != ITPP_OK) return st;
    }
  }
  // results
  std::vector<double> dth((size_t)std::max<int64_t>(Gtot, 1), 0.0);
  if (Gtot > 0)
    HIP_TRY(c, hipMemcpyAsync(dth.data(), B.dtheta, sizeof(double) * Gtot, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, restore_snapshot(c, SF));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  st = check_error(c);
  if (st != ITPP_OK) return st;
  const int G = (int)c->glist.size();
  std::vector<HostSum> da(c->terms.size());
  HostSum dd;
  for (int64_t g = 0; g < Gtot; ++g) {
    const int sg = c->glist[(int)(g % G)];
    const int k = c->sched_term[sg];
    const double mlt = c->sched_mult[sg];
    da[k].add(mlt * c->fwd_dtau * dth[g]);
    dd.add(c->terms[k].alpha * mlt * dth[g]);
  }
  for (size_t k = 0; k < da.size(); ++k) d_alpha[k] = da[k].value();
  *d_dtau = dd.value();
  if (d_theta)
    for (int64_t g = 0; g < Gtot; ++g) d_theta[g] = dth[g];
  return ITPP_OK;
}

}  // namespace

extern "C" {

itpp_status itpp_set_adjoint(itpp_ctx c, int32_t every_steps, int64_t workspace_bytes) {
  if (!c) return ITPP_ERR_ARG;
  if (every_steps < 0 || workspace_bytes < 0) return fail(c, ITPP_ERR_ARG, "negative argument");
  if (every_steps > 0 && c->f32) return fail(c, ITPP_ERR_ARG, "the reverse sweep needs ITPP_F64 coefficients");
  if (every_steps > 0 && c->max_weight > 0) return fail(c, ITPP_ERR_STATE, "the reverse sweep has no weight cutoff");
  c->ckpt_every = every_steps;
  c->adj_workspace = workspace_bytes;
  free_ckpts(c);
  c->fwd_valid = c->fwd_gates == 0;
  return ITPP_OK;
}

itpp_status itpp_num_gates(itpp_ctx c, int64_t* out) {
  if (!c || !out) return ITPP_ERR_ARG;
  *out = c->fwd_gates;
  return ITPP_OK;
}

itpp_status itpp_backward(itpp_ctx c, int32_t m, const uint64_t* x, const uint64_t* z, const double* coef,
                          double* value, double* d_alpha, double* d_dtau, double* d_theta, int64_t d_theta_capacity) {
  if (!c) return ITPP_ERR_ARG;
  if (!value || !d_alpha || !d_dtau) return fail(c, ITPP_ERR_ARG, "null output");
  if (d_theta && d_theta_capacity < c->fwd_gates)
    return fail(c, ITPP_ERR_ARG, "d_theta capacity is smaller than the number of gates (itpp_num_gates)");
  if (m < 0 || (m > 0 && (!x || !z || !coef))) return fail(c, ITPP_ERR_ARG, "bad observable arrays");
  if (!c->ready) return fail(c, ITPP_ERR_STATE, "no valid state (reset required)");
  if (c->f32) return fail(c, ITPP_ERR_ARG, "the reverse sweep needs ITPP_F64 coefficients");
  if (c->ckpt_every <= 0 || !c->fwd_valid || (c->ckpts.empty() && c->fwd_gates > 0))
    return fail(c, ITPP_ERR_STATE, "no replayable forward run: call itpp_set_adjoint, reset, then evolve with one dtau");
  const int W = c->W;
  for (int j = 0; j < m; ++j)
    for (int q = 0; q < W; ++q) {
      const int hi = c->n - 64 * q;
      if (hi < 64) {
        const uint64_t bad = hi <= 0 ? ~0ull : ~((1ull << hi) - 1ull);
        if ((x[(size_t)j * W + q] | z[(size_t)j * W + q]) & bad)
          return fail(c, ITPP_ERR_ARG, "observable has bits at or above n_qubits");
      }
    }
  itpp_status st = check_error(c);
  if (st != ITPP_OK) return st;
  const bool timing = c->timing;
  c->timing = false;
  const int64_t Gtot = c->fwd_gates;
  std::vector<void*> mem;
  auto take = [&](uint64_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<uint64_t>(bytes, 256)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    mem.push_back(p);
    return p;
  };
  AdjBuffers B{};
  B.lam[0] = static_cast<double*>(take(c->cap * sizeof(double)));
  B.lam[1] = static_cast<double*>(take(c->cap * sizeof(double)));
  B.sdev = static_cast<double*>(take(2 * sizeof(double)));
  B.part = static_cast<double*>(take(4 * c->status_cap * sizeof(double)));
  B.ntiles = static_cast<uint64_t*>(take(sizeof(uint64_t)));
  B.dtheta = static_cast<double*>(take(std::max<int64_t>(Gtot, 1) * sizeof(double)));
  uint64_t* dx = static_cast<uint64_t*>(take(sizeof(uint64_t) * std::max(m, 1) * W));
  uint64_t* dz = static_cast<uint64_t*>(take(sizeof(uint64_t) * std::max(m, 1) * W));
  double* dc = static_cast<double*>(take(sizeof(double) * std::max(m, 1)));
  Arena ar;
  bool ok = B.lam[0] && B.lam[1] && B.sdev && B.part && B.ntiles && B.dtheta && dx && dz && dc;
  if (ok) {
    uint64_t want = (uint64_t)c->adj_workspace;
    if (want == 0) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) == hipSuccess) want = (uint64_t)(0.7 * (double)fr);
    }
    ar.base = static_cast<uint8_t*>(take(want));
    ar.size = want;
    ok = ar.base != nullptr;
  }
  hipError_t ce = hipSuccess;
  if (ok && m > 0) {
    ce = hipMemcpyAsync(dx, x, sizeof(uint64_t) * m * W, hipMemcpyHostToDevice, c->stream);
    if (ce == hipSuccess) ce = hipMemcpyAsync(dz, z, sizeof(uint64_t) * m * W, hipMemcpyHostToDevice, c->stream);
    if (ce == hipSuccess) ce = hipMemcpyAsync(dc, coef, sizeof(double) * m, hipMemcpyHostToDevice, c->stream);
  }
  if (!ok) {
    st = fail(c, ITPP_ERR_OOM, "device memory for the reverse sweep is not available");
  } else if (ce != hipSuccess) {
    st = hip_fail(c, ce, "copy of the observable to the device");
  } else {
    double v = 0.0;
    st = backward_impl(c, m, dx, dz, dc, &v, d_alpha, d_dtau, d_theta, ar, B);
    if (st == ITPP_OK) *value = v;
  }
  (void)hipStreamSynchronize(c->stream);
  for (void* p : mem) (void)hipFree(p);
  c->timing = timing;
  if (st != ITPP_OK) c->ready = false;
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches of independent instances.

struct itpp_batch_s {
  std::vector<itpp_ctx> inst;
  void* arena = nullptr;
  int32_t workers = 4;
  std::string err;
};

namespace {

itpp_status batch_fail(itpp_batch b, itpp_status s, const std::string& m) {
  if (b) b->err = m;
  return s;
}

// Run fn(i) for every instance on `workers` host threads; instances are
// taken largest-work first from a shared counter.  Returns the first error.
template <typename F>
itpp_status batch_run(itpp_batch b, const std::vector<double>& work, int workers, F fn) {
  const int n = (int)b->inst.size();
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  std::atomic<int> next{0};
  std::vector<itpp_status> res(n, ITPP_OK);
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto body = [&]() {
    (void)hipSetDevice(dev);
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      res[order[k]] = fn(order[k]);
    }
  };
  const int nt = std::max(1, std::min(workers, n));
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(body);
  body();
  for (auto& t : th) t.join();
  for (int i = 0; i < n; ++i)
    if (res[i] != ITPP_OK)
      return batch_fail(b, res[i], "instance " + std::to_string(i) + ": " + b->inst[i]->err);
  return ITPP_OK;
}

}  // namespace

extern "C" {

itpp_status itpp_batch_create(int32_t n_inst, const itpp_config* cfgs, itpp_batch* out) {
  if (!cfgs || !out || n_inst < 1) return create_fail(ITPP_ERR_ARG, "bad batch arguments");
  for (int i = 0; i < n_inst; ++i) {
    itpp_status s = check_config(&cfgs[i]);
    if (s != ITPP_OK) return s;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  itpp_status s = device_props(&dev, &prop);
  if (s != ITPP_OK) return s;
  std::vector<uint64_t> bytes(n_inst);
  uint64_t total = 0;
  for (int i = 0; i < n_inst; ++i) {
    s = create_impl(&cfgs[i], dev, prop, nullptr, 0, &bytes[i], nullptr);
    if (s != ITPP_OK) return s;
    total += bytes[i];
  }
  itpp_batch b = new (std::nothrow) itpp_batch_s;
  if (!b) return ITPP_ERR_OOM;
  if (hipMalloc(&b->arena, total) != hipSuccess) {
    (void)hipGetLastError();
    delete b;
    return create_fail(ITPP_ERR_OOM, "batch arena of " + std::to_string(total) + " bytes is not available");
  }
  uint64_t off = 0;
  for (int i = 0; i < n_inst; ++i) {
    itpp_config cfg = cfgs[i];
    hipStream_t st = nullptr;
    if (hipStreamCreate(&st) != hipSuccess) {
      (void)hipGetLastError();
      itpp_batch_destroy(b);
      return create_fail(ITPP_ERR_DEVICE, "hipStreamCreate failed");
    }
    cfg.stream = st;
    itpp_ctx c = nullptr;
    s = create_impl(&cfg, dev, prop, static_cast<uint8_t*>(b->arena) + off, bytes[i], nullptr, &c);
    if (s != ITPP_OK) {
      (void)hipStreamDestroy(st);
      itpp_batch_destroy(b);
      return s;
    }
    c->own_stream = st;
    b->inst.push_back(c);
    off += bytes[i];
  }
  *out = b;
  return ITPP_OK;
}

itpp_status itpp_batch_destroy(itpp_batch b) {
  if (!b) return ITPP_OK;
  for (itpp_ctx c : b->inst) itpp_destroy(c);
  if (b->arena) (void)hipFree(b->arena);
  delete b;
  return ITPP_OK;
}

itpp_ctx itpp_batch_instance(itpp_batch b, int32_t i) {
  if (!b || i < 0 || i >= (int32_t)b->inst.size()) return nullptr;
  return b->inst[i];
}

itpp_status itpp_batch_set_workers(itpp_batch b, int32_t workers) {
  if (!b) return ITPP_ERR_ARG;
  if (workers < 1 || workers > 64) return batch_fail(b, ITPP_ERR_ARG, "workers must be in 1..64");
  b->workers = workers;
  return ITPP_OK;
}

itpp_status itpp_batch_evolve(itpp_batch b, const double* dtau, const int64_t* n_steps, itpp_stats* st) {
  if (!b || !dtau || !n_steps) return ITPP_ERR_ARG;
  const int n = (int)b->inst.size();
  std::vector<double> work(n);
  for (int i = 0; i < n; ++i) work[i] = (double)n_steps[i] * (double)b->inst[i]->glist.size() * b->inst[i]->n;
  return batch_run(b, work, b->workers, [&](int i) {
    return itpp_evolve(b->inst[i], dtau[i], n_steps[i], st ? &st[i] : nullptr);
  });
}

itpp_status itpp_batch_autotune(itpp_batch b, const double* dtau, int64_t warm_gates, int64_t probe_gates,
                                int32_t* best_shape, int32_t* best_workers, int32_t* best_grid_div,
                                double* best_rate) {
  if (!b || !dtau || warm_gates < 0 || probe_gates < 1) return ITPP_ERR_ARG;
  const int n = (int)b->inst.size();
  std::vector<double> work(n);
  for (int i = 0; i < n; ++i) work[i] = (double)b->inst[i]->n;
  // one setting: gate shapes (one for n <= 64, one above), workers, grid divisor
  struct Setting {
    int s_small, s_large, workers, grid_div;
  };
  auto apply = [&](const Setting& x) -> itpp_status {
    for (itpp_ctx c : b->inst) {
      c->shape = c->NW == 4 ? x.s_large : x.s_small;
      c->grid_div = x.grid_div;
      drop_step_graph(c);
      itpp_status s = itpp_reset(c);
      if (s != ITPP_OK) return batch_fail(b, s, c->err);
    }
    return ITPP_OK;
  };
  auto probe = [&](const Setting& x, double* rate) -> itpp_status {
    itpp_status s = apply(x);
    if (s != ITPP_OK) return s;
    s = batch_run(b, work, x.workers, [&](int i) { return itpp_evolve_gates(b->inst[i], dtau[i], warm_gates, nullptr); });
    if (s != ITPP_OK) return s;
    std::vector<itpp_stats> st(n);
    const auto t0 = std::chrono::steady_clock::now();
    s = batch_run(b, work, x.workers, [&](int i) { return itpp_evolve_gates(b->inst[i], dtau[i], probe_gates, &st[i]); });
    if (s != ITPP_OK) return s;
    const double dt = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    double tu = 0.0;
    for (const auto& y : st) tu += y.term_updates;
    *rate = dt > 0.0 ? tu / dt : 0.0;
    return ITPP_OK;
  };
  // coordinate descent: the shape pair first, then workers, then the grid
  Setting best{1, 1, b->workers, 1};
  double best_r = -1.0;
  auto consider = [&](const Setting& x) -> itpp_status {
    double r = 0.0;
    itpp_status s = probe(x, &r);
    if (s != ITPP_OK) return s;
    if (r > best_r) {
      best_r = r;
      best = x;
    }
    return ITPP_OK;
  };
  const Setting start = best;
  for (int ss = 0; ss < 3; ++ss)
    for (int sl = 0; sl < 3; ++sl) {
      itpp_status s = consider(Setting{ss, sl, start.workers, start.grid_div});
      if (s != ITPP_OK) return s;
    }
  const Setting after_shapes = best;
  for (int w : {2, 4, 8, 16}) {
    if (w == after_shapes.workers) continue;
    itpp_status s = consider(Setting{after_shapes.s_small, after_shapes.s_large, w, after_shapes.grid_div});
    if (s != ITPP_OK) return s;
  }
  const Setting after_workers = best;
  for (int g : {2, 4, 8}) {
    itpp_status s = consider(Setting{after_workers.s_small, after_workers.s_large, after_workers.workers, g});
    if (s != ITPP_OK) return s;
  }
  itpp_status s = apply(best);
  if (s != ITPP_OK) return s;
  b->workers = best.workers;
  if (best_shape) *best_shape = best.s_small + 3 * best.s_large;
  if (best_workers) *best_workers = best.workers;
  if (best_grid_div) *best_grid_div = best.grid_div;
  if (best_rate) *best_rate = best_r;
  return ITPP_OK;
}

const char* itpp_batch_last_error(itpp_batch b) {
  if (!b) return g_create_error.c_str();
  return b->err.c_str();
}

}  // extern "C"
