// Internal structures shared by the ITPP kernels and the host runtime.
//
// State layout in HBM (one "side" of a ping-pong pair):
//   key words  kw[0..NW-1][cap]   (structure of arrays, NW = 2W uint64 words)
//   coef       coef[cap]          (double, value before normalisation)
// Keys are stored in a bit-permuted representation ("rep"): the 2n x/z bits
// of a string are placed at positions chosen by the host so that the bits
// flipped by the NEXT gate are the most significant ones.  Numeric order of
// rep keys is then a lexicographic bit order in which the strings of equal
// flip-bit pattern ("class") are contiguous, and xor with the gate string
// only changes the class.  The pairing P <-> Q P of Eq. (ITPP_PropRules)
// becomes a merge-join of class c with class ~c.
//
// A stored state is a set of regions (c, e): c = class under the gate that
// produced it, e = class under the gate that will read it.  The reader sees
// its class e as the concatenation over c of regions (c, e), which is sorted.
#pragma once
#include <cstddef>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace itpp {

constexpr int kMaxClassBits = 2;            // a gate may flip at most two key bits
constexpr int kMaxClasses = 1 << kMaxClassBits;
constexpr int kMaxWords = 2;                 // W <= 2  (n <= 128)
constexpr int kMaxKeyWords = 2 * kMaxWords;  // NW <= 4
constexpr int kMaxBits = 64 * kMaxKeyWords;  // 256
constexpr int kHistBins = 1024;              // |c| histogram: 16 bins per octave
constexpr int kHistShift = 48;               // bits >> 48: 11 exponent + 4 mantissa bits
constexpr uint32_t kHistBase = (1023u - 62u) << 4;  // bin 0 starts at 2^-62
constexpr int kFineBins = 1024;              // fine |c| histogram around the predicted K-th value
constexpr int kFineShift = 38;               // bin width 2^38 ulps of the f64 pattern
constexpr uint64_t kFineHalf = 1ull << 47;   // window half width (~2.2% relative)
constexpr int kRatioSlots = 1024;            // schedule positions with a recorded K-th value ratio
constexpr uint32_t kStatusClearEvery = 2048; // look-back tags are 12-bit epochs (4095 values)

// Description of a stored state (written by the gate that produced it).
struct Plan {
  uint32_t cnt[kMaxClasses][kMaxClasses];   // elements written in region (c, e)
  uint64_t base[kMaxClasses][kMaxClasses];  // first element of region (c, e)
  uint32_t ncnt[kMaxClasses][kMaxClasses];  // stored elements of class e with pattern f of the gate after
  int32_t wc;                               // class bits of the producer (c)
  int32_t we;                               // class bits of the reader (e)
  uint32_t pad[2];
};

// Truncation / normalisation decided after a gate, applied when the next
// gate (or a readout) loads the stored elements.
struct Filter {
  double cI;                 // identity coefficient before normalisation
  uint64_t kth_bits;         // |c| bit pattern of the (K-1)-th largest non-identity
  uint32_t cap_active;       // 1: elements below kth_bits are dropped
  uint32_t tie_active;       // 1: elements equal to kth_bits are kept only up to tie_key
  uint64_t tie_key[kMaxKeyWords];  // canonical key (x words, then z words) of the last tied survivor
  uint64_t n_written;        // stored elements (identity included)
  uint64_t n_survivors;      // elements that pass the filter
  uint64_t ref_bits;         // |c| bits near which the next gate's K-th value is expected (0: none)
};

// The epoch after e (skips 0; the wrap lands on a multiple of
// kStatusClearEvery, so the records are cleared before the next use).
__host__ __device__ inline uint32_t next_epoch(uint32_t e) { return e + 1u == 0u ? kStatusClearEvery : e + 1u; }

// Per-run control block (device).
struct Ctl {
  // The tile ticket of the running gate, alone in its 128-byte line: every
  // tile takes one with a device-scope atomic, and other traffic to the same
  // line would queue behind those atomics.
  uint32_t ticket;
  uint32_t pad_ticket[31];
  // Read by every workgroup when it starts (one line).
  uint32_t error;            // sticky error code (see kErr*)
  uint32_t halt;             // 1: a speculative gate must be redone; later kernels do nothing
  // Look-back tag of the running gate and its serial number: advanced on the
  // device once per gate attempt (select_decide, adj_reduce_kernel), so the
  // launches of a gate carry no per-launch arguments and a recorded graph
  // of a Trotter step can be replayed.  The look-back records are cleared
  // whenever the epoch is a multiple of kStatusClearEvery (partition_kernel);
  // it starts at kStatusClearEvery and is never 0, the tag of a cleared record.
  uint32_t epoch;
  uint32_t pad_epoch;
  uint64_t gate_serial;
  uint64_t halt_serial;      // serial of the gate that asked to be redone
  uint32_t pad_read[24];
  // Added to by workgroups when they finish.
  uint64_t n_written_nonid;  // written non-identity outputs of the running gate
  uint64_t n_above_hi;       // written non-identity outputs above the fine window
  double cI_out;             // identity output of the running gate
  uint32_t have_cI;
  uint32_t pad_cnt[25];
  uint32_t hist[kHistBins];
  uint32_t fhist[kFineBins];
  // selection scratch
  uint64_t sel_lo, sel_hi;   // |c| bit range that holds the K-th value
  uint32_t sel_need;         // elements still needed from that range
  uint32_t pad2;
  uint64_t cand_count;
  uint32_t need_coarse;      // the fine window missed: select from a full histogram
  uint32_t hist_done;        // workgroups of the full histogram that have finished
  uint32_t pad3;
  double term_updates;
  double alg_elems;          // sum over gates of survivors in + survivors out
  uint64_t gates;
  uint32_t cap_hit;
  uint64_t spec_gates;       // gates that ran with a speculative write threshold
  double written_elems;      // sum over gates of the strings stored (identity included)
  // over the gates since the host last set them (run statistics):
  double cI_min, cI_max;     // identity coefficient before normalisation
  double kth_min;            // smallest normalised K-th |c| of a gate whose cap bound
  // per schedule position: the exact K-th value of the gate's output over the
  // value predicted from its input (the last time that position ran; 0: none)
  float kth_ratio[kRatioSlots];
};
static_assert(offsetof(Ctl, error) == 128 && offsetof(Ctl, n_written_nonid) == 256 && offsetof(Ctl, hist) == 384,
              "the ticket, the start-of-workgroup reads and the end-of-workgroup counters have a line each");

enum : uint32_t {
  kErrNone = 0,
  kErrNumeric = 1,     // identity coefficient not finite / not positive
  kErrCapacity = 2,    // a buffer bound was exceeded (library bug or bad sizing)
  kErrSpin = 3,        // a look-back wait exceeded its bound
  kErrCap = 4,         // cap reached under the FAIL policy
  kErrPhase = 5,       // commuting strings gave an imaginary phase
};

// Look-back records, as dense word arrays of n = status_cap entries each (so
// that 64 consecutive tiles are one coalesced load): word array s (s = 0, 1)
// at [s*n, s*n + n) packs a tile's output counts of stream s (class cA / cB
// of the join) for the 4 next classes as 12-bit fields (bits 0..47), a
// 12-bit epoch tag (bits 52..63) and, in bit 48, a flag set once the
// inclusive prefix is published; word array 2 + q holds the inclusive prefix
// of counter q as (epoch << 32) | count.  Every word validates itself, so
// single relaxed atomic loads suffice.
constexpr int kStatusWords = 2 + 2 * kMaxClasses;
typedef unsigned long long TileStatus;

// Device arrays of one side of the ping-pong state buffers.
// coef points to binary64 or binary32 values (the context's precision).
struct Side {
  uint64_t* kw[kMaxKeyWords];
  void* coef;
};

// Rep positions of the canonical bits of a stored state.
struct RepPos {
  uint8_t pos[kMaxBits];
  int32_t nbits;
  int32_t pad;
};

// Parameters of one elementary gate, computed on the host.
struct GateParams {
  double ch, sh;             // cosh(theta), sinh(theta)
  int32_t nbits;             // 2n: meaningful rep bits
  int32_t w;                 // class bits of this gate (1 or 2)
  int32_t w1;                // class bits of the next gate
  int32_t w2;                // class bits of the gate after next
  uint64_t cmask[kMaxKeyWords];  // rep positions whose parity marks anticommutation
  // phase of Q P for commuting P: qubits in the support of Q
  int32_t nsup;
  int32_t aQ;                // number of Y letters in Q (mod 4)
  int32_t px[2], pz[2];      // rep positions of x_j, z_j
  int32_t qx[2], qz[2];      // letters of Q on those qubits
  int32_t mv[kMaxClassBits];     // rep positions (sequential) moved to the top for the next gate
  int32_t fpos[kMaxClassBits];   // positions, in the next rep, of the bits of the gate after next
  int32_t ov;                // pattern over the next gate's bits flipped by this gate
  int32_t epos[kMaxClassBits];   // positions, in this rep, of the next gate's flip bits (class bits)
  int32_t fposg[kMaxClassBits];  // positions, in this rep, of the flip bits of the gate after next
  int32_t ovf;               // pattern over the latter bits flipped by this gate
  int32_t spec;              // 1: write only outputs above a margin below the predicted K-th value
  int32_t spos;              // schedule position (index of kth_ratio), -1: none
  uint64_t qm1[kMaxKeyWords];    // this gate's flip mask in the next rep (branch key = self key ^ qm1)
  uint64_t topm[kMaxKeyWords];   // this gate's flip mask in the current rep (the w top bits)
  int32_t wmax;              // Pauli-weight cutoff (0: none)
  int32_t pad_wmax;
  uint64_t wtab;             // weight(Q P) - weight(P) + 2 for the 16 support patterns (3 bits each)
  double spec_mult;          // that margin as a factor of the predicted value
  int32_t tile;              // merged elements per tile
  uint32_t check_write_threshold;
  double delta;              // keep |c| > delta
  uint64_t cap_elems;        // capacity of each side in elements
  uint64_t status_cap;       // entries of the look-back status array
  // Rep positions packed one per byte, for the layer kernel (computed once
  // per gate on the host):
  uint32_t mvpos;    // mv[0] | mv[1] << 8 (sequential positions of the next gate's flip bits)
  uint32_t fgpos;    // fposg[0] | fposg[1] << 8 | epos[0] << 16 | epos[1] << 24
  uint32_t phpos;    // x_j0 | z_j0 << 8 | x_j1 << 16 | z_j1 << 24 (support of Q, current rep)
  uint32_t q1pos;    // this gate's flip bits in the next rep (w bytes)
  uint32_t etab;     // e mod 4 of Q P = i^e R for the 16 patterns of the phase bits (2 bits each)
  uint32_t lflags;   // ov | ovf << 2 | w2 << 4 | nph << 6 | phflip << 9
  uint8_t pos_in[kMaxBits];  // canonical bit -> rep position of the stored (input) keys
};

// Reverse-sweep arguments of the adjoint gate kernel (FP64 states only).
struct AdjArgs {
  const double* lam_out;    // lambda' = dL/da', parallel to the packed output of the gate
  double* lam_in;           // lambda = dL/da for the gate's input (same positions as the input)
  const Plan* plan_next;    // packed plan of the output
  const Filter* filt_next;  // filter decided after the gate (its cI is b_I)
  const double* s_in;       // sum of lambda' a' over the kept output
  double* part;             // 4 doubles per tile: dtheta sum, compensation, sum lambda a, compensation
  uint64_t* ntiles;         // tiles of the launch (written by the kernel)
  uint64_t lam_out_len;     // elements of lam_out
};

// Selection scratch (device): candidates of the K-th value and tied keys.
struct SelBuf {
  uint64_t* cand_bits;
  uint64_t* cand_idx;
  uint64_t* tie_keys;   // kMaxKeyWords words per tied element
  uint64_t cap;         // capacity of each array in elements
};

// Host launchers (gate and partition in itpp_gate.hip, the others in
// itpp_kernels.hip).
hipError_t launch_init(int nw, int f32, Side s0, Plan* plan, Filter* filt, Ctl* ctl, int w0, hipStream_t st);
hipError_t launch_partition(int nw, const GateParams& gp, Side in, const Plan* plan_in, Ctl* ctl, uint64_t* part,
                            TileStatus* status, hipStream_t st);
hipError_t launch_gate(int nw, int f32, int shape, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                       Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part,
                       int grid, hipStream_t st);
// The same gate under the real-time rule (gp.ch = cos, gp.sh = sin).
hipError_t launch_gate_rt(int nw, int f32, int shape, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                       Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part,
                       int grid, hipStream_t st);
hipError_t launch_select(int nw, int f32, Side out, const Plan* plan_out, const Filter* filt_in,
                         Filter* filt_out, Plan* plan_next, Ctl* ctl, SelBuf sel, const RepPos& rp,
                         int64_t K, int cap_fail, int spec, int spos, int grid, hipStream_t st);
hipError_t launch_prepare(Plan* plan_out, Ctl* ctl, hipStream_t st);
hipError_t launch_adjoint_gate(int nw, const GateParams& gp, Side in, const Plan* plan_in, Plan* plan_scratch,
                               const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part,
                               const AdjArgs& adj, int grid, hipStream_t st);
hipError_t launch_adj_reduce(const double* part, const uint64_t* ntiles, double* dtheta_out, double* s_out,
                             Ctl* ctl, hipStream_t st);
hipError_t launch_pack(int nw, int f32, Side src, const Plan* plan_src, Side dst, Plan* plan_dst, int grid,
                       hipStream_t st);
hipError_t launch_seed(int nw, Side s, const Plan* plan, const Filter* filt, const RepPos& rp, const uint64_t* ox,
                       const uint64_t* oz, const double* oc, int32_t m, double* lam, hipStream_t st);
hipError_t launch_observe(int nw, int f32, Side s, const Plan* plan, const Filter* filt, const RepPos& rp,
                          const uint64_t* ox, const uint64_t* oz, const double* oc, int32_t m,
                          double* result, Ctl* ctl, hipStream_t st);
hipError_t launch_export(int nw, int f32, Side s, const Plan* plan, const Filter* filt, const RepPos& rp,
                         uint64_t* ex, uint64_t* ez, double* ec, unsigned long long* count,
                         uint64_t limit, int grid, hipStream_t st);
// The layer kernel (itpp_layer.hip): the forward gate with small workgroups,
// several per CU (see launch_layer).
hipError_t launch_layer(int nw, int f32, bool rt, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                        Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part, int cus,
                        hipStream_t st);
int layer_tile();
int gate_tile(int nw, int shape);
int gate_min_tile(int nw);
int gate_wgs_per_cu(int shape);

}  // namespace itpp
