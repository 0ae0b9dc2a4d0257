// Device-side types and helpers shared by the ITPP kernels (gfx950, wave64):
// bit-permuted Pauli keys, coefficient arithmetic of the two storage
// precisions, the deferred filter, class views of a stored state and the
// join layout of a gate.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "itpp_internal.h"

namespace itpp {

template <int NW>
struct Key {
  uint64_t w[NW];
};

template <int NW>
__device__ __forceinline__ bool key_less(const Key<NW>& a, const Key<NW>& b) {
#pragma unroll
  for (int i = NW - 1; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i];
  return false;
}

template <int NW>
__device__ __forceinline__ bool key_eq(const Key<NW>& a, const Key<NW>& b) {
  bool e = true;
#pragma unroll
  for (int i = 0; i < NW; ++i) e = e && (a.w[i] == b.w[i]);
  return e;
}

template <int NW>
__device__ __forceinline__ bool key_zero(const Key<NW>& a) {
  uint64_t o = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) o |= a.w[i];
  return o == 0;
}

// Bit access at a runtime position without indexing the register array
// (a dynamic index would move the key to scratch memory).
template <int NW>
__device__ __forceinline__ uint64_t word_at(const Key<NW>& k, int wi) {
  uint64_t v = k.w[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) v = (wi == i) ? k.w[i] : v;
  return v;
}

template <int NW>
__device__ __forceinline__ int get_bit(const Key<NW>& k, int p) {
  return (int)((word_at(k, p >> 6) >> (p & 63)) & 1ull);
}

template <int NW>
__device__ __forceinline__ void xor_bit(Key<NW>& k, int p, uint64_t v) {
  const int wi = p >> 6;
  const uint64_t m = v << (p & 63);
#pragma unroll
  for (int i = 0; i < NW; ++i) k.w[i] ^= (wi == i) ? m : 0ull;
}

template <int NW>
__device__ __forceinline__ void flip_bit(Key<NW>& k, int p) {
  xor_bit(k, p, 1ull);
}

// Flip the w most significant meaningful bits (the bits the gate flips).
template <int NW>
__device__ __forceinline__ Key<NW> xor_top(Key<NW> k, int nbits, int w) {
  for (int b = nbits - w; b < nbits; ++b) flip_bit(k, b);
  return k;
}

// Key xor a uniform mask (a gate's flip bits, precomputed per gate).
template <int NW>
__device__ __forceinline__ Key<NW> xor_mask(Key<NW> k, const uint64_t* m) {
#pragma unroll
  for (int i = 0; i < NW; ++i) k.w[i] ^= m[i];
  return k;
}

// Class = pattern of the w most significant meaningful bits.
template <int NW>
__device__ __forceinline__ int class_of(const Key<NW>& k, int nbits, int w) {
  int c = 0;
  for (int b = 0; b < w; ++b) c |= get_bit(k, nbits - w + b) << b;
  return c;
}

// Move the bit at position p to position nbits-1; bits above p shift down.
template <int NW>
__device__ __forceinline__ Key<NW> move_top(const Key<NW>& k, int p, int nbits) {
  const uint64_t b = (uint64_t)get_bit(k, p);
  Key<NW> r;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    uint64_t shr = (k.w[i] >> 1) | ((i + 1 < NW) ? (k.w[i + 1] << 63) : 0ull);
    const int lo = 64 * i;
    uint64_t lm;
    if (p <= lo)
      lm = 0ull;
    else if (p >= lo + 64)
      lm = ~0ull;
    else
      lm = (1ull << (p - lo)) - 1ull;
    r.w[i] = (k.w[i] & lm) | (shr & ~lm);
  }
  xor_bit(r, nbits - 1, b);  // bit nbits-1 of the shifted key is zero
  return r;
}

// Bit p (a uniform rep position) of a key.
template <int NW>
__device__ __forceinline__ uint32_t bit_at(const Key<NW>& k, uint32_t p) {
  return (uint32_t)(word_at(k, (int)(p >> 6)) >> (p & 63u)) & 1u;
}

template <int NW>
__device__ __forceinline__ void flip_at(Key<NW>& k, uint32_t p) {
  const uint64_t m = 1ull << (p & 63u);
  const int wi = (int)(p >> 6);
#pragma unroll
  for (int i = 0; i < NW; ++i) k.w[i] ^= (wi == i) ? m : 0ull;
}

// Move the bit at rep position p to the top position top; the bits above p
// shift down by one.  b receives the bit.
template <int NW>
__device__ __forceinline__ Key<NW> move_bit(const Key<NW>& k, uint32_t p, uint32_t top, uint32_t& b) {
  b = bit_at(k, p);
  Key<NW> r;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint32_t lo = 64u * (uint32_t)i;
    const uint64_t lm = p >= lo + 64u ? ~0ull : (p <= lo ? 0ull : (1ull << (p - lo)) - 1ull);
    const uint64_t s = (k.w[i] >> 1) | ((i + 1 < NW) ? (k.w[i + 1] << 63) : 0ull);
    r.w[i] = (k.w[i] & lm) | (s & ~lm);
  }
  const uint64_t t = (uint64_t)b << (top & 63u);
  const int twi = (int)(top >> 6);
#pragma unroll
  for (int i = 0; i < NW; ++i) r.w[i] |= (twi == i) ? t : 0ull;
  return r;
}

// Count one output in the 16 (class, next-next class) bins, 16-bit fields.
__device__ __forceinline__ void bin_add(uint64_t (&nb)[4], int bin) {
  const uint64_t inc = 1ull << (16 * (bin & 3));
  const int wsel = bin >> 2;
#pragma unroll
  for (int i = 0; i < 4; ++i) nb[i] += (wsel == i) ? inc : 0ull;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <int NW>
__device__ __forceinline__ Key<NW> load_key(const Side& s, uint64_t i) {
  Key<NW> k;
#pragma unroll
  for (int w = 0; w < NW; ++w) k.w[w] = s.kw[w][i];
  return k;
}

template <int NW>
__device__ __forceinline__ void store_key(const Side& s, uint64_t i, const Key<NW>& k) {
#pragma unroll
  for (int w = 0; w < NW; ++w) s.kw[w][i] = k.w[w];
}

// Canonical key (x words then z words) of a rep key.
template <int NW>
__device__ inline Key<NW> to_canonical(const Key<NW>& k, const uint8_t* pos, int nbits) {
  Key<NW> c;
#pragma unroll
  for (int i = 0; i < NW; ++i) c.w[i] = 0;
  const int n = nbits / 2;
  constexpr int W = NW / 2;
  for (int cb = 0; cb < nbits; ++cb) {
    if (get_bit(k, pos[cb])) {
      const int word = (cb < n) ? (cb >> 6) : (W + ((cb - n) >> 6));
      const int bit = (cb < n) ? (cb & 63) : ((cb - n) & 63);
      xor_bit(c, 64 * word + bit, 1ull);
    }
  }
  return c;
}

// Canonical order: x words from the most significant, then z words.
template <int NW>
__device__ inline bool canon_le(const Key<NW>& a, const Key<NW>& b) {
  constexpr int W = NW / 2;
  for (int i = W - 1; i >= 0; --i)
    if (a.w[i] != b.w[i]) return a.w[i] < b.w[i];
  for (int i = W - 1; i >= 0; --i)
    if (a.w[W + i] != b.w[W + i]) return a.w[W + i] < b.w[W + i];
  return true;
}

__device__ __forceinline__ uint64_t abs_bits(double v) {
  return (uint64_t)__double_as_longlong(v) & 0x7fffffffffffffffull;
}

// Coefficient arithmetic of the two storage precisions.  Products and sums
// are rounded to the storage type T; the division by the identity
// coefficient is done in double and rounded once to T; magnitudes are
// compared, histogrammed and selected as doubles (exact widening, so the
// order is that of T).
__device__ __forceinline__ double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double abs_d(double v) { return fabs(v); }
__device__ __forceinline__ double abs_d(float v) { return (double)fabsf(v); }
template <typename T>
__device__ __forceinline__ T normalised(T c, double cI) {
  return (T)((double)c / cI);
}
template <typename T>
__device__ __forceinline__ T* coefs(const Side& s) {
  return static_cast<T*>(s.coef);
}

// Error-free sum (Knuth TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = __dadd_rn(a, b);
  const double bb = __dsub_rn(s, a);
  e = __dadd_rn(__dsub_rn(a, __dsub_rn(s, bb)), __dsub_rn(b, bb));
}


__device__ __forceinline__ int hist_bin(uint64_t bits) {
  const int64_t b = (int64_t)(bits >> kHistShift) - (int64_t)kHistBase;
  return b < 0 ? 0 : (b >= kHistBins ? kHistBins - 1 : (int)b);
}

// The K-th value a gate's output is expected to have (before the gate's own
// normalisation): the previous gate's exact K-th value, normalised, times
// the ratio recorded at this schedule position the last time it ran (the
// K-th value drifts slowly with beta); 0 when there is no previous K-th
// value.  raw receives the prediction without the ratio.
__device__ inline double predicted_kth(const Filter& fin, int spos, const Ctl* ctl, double* raw,
                                       bool* have_ratio = nullptr) {
  if (have_ratio) *have_ratio = false;
  if (!fin.ref_bits) {
    if (raw) *raw = 0.0;
    return 0.0;
  }
  const double pred = __longlong_as_double((long long)fin.ref_bits) / fin.cI;
  if (raw) *raw = pred;
  if (spos < 0) return pred;
  const float r = ctl->kth_ratio[spos];
  if (!(r > 0.f)) return pred;
  if (have_ratio) *have_ratio = true;
  return __dmul_rn(pred, (double)r);
}

// Whether a gate writes only the outputs above a margin below its predicted
// K-th value: speculation is allowed, the cap bound after the previous gate,
// and this schedule position has a recorded ratio (from the second capped
// Trotter step on; before that the K-th value still moves fast).  The gate
// kernels and select_decide take the same decision.
__device__ inline bool gate_speculates(const Filter& fin, int spec, int spos, const Ctl* ctl) {
  bool have_ratio = false;
  (void)predicted_kth(fin, spos, ctl, nullptr, &have_ratio);
  return spec && fin.cap_active && have_ratio;
}

// Fine-histogram window around the predicted K-th value, and the write
// threshold: delta, raised to a margin below the prediction when the gate
// speculates.
__device__ inline void gate_window(const Filter& fin, const GateParams& gp, const Ctl* ctl, uint64_t& win_lo,
                                   uint64_t& win_hi, double& tw) {
  win_lo = win_hi = 0;
  tw = gp.delta;
  const double pred = predicted_kth(fin, gp.spos, ctl, nullptr);
  if (pred > 0.0) {
    const uint64_t cb = abs_bits(pred);
    win_lo = cb > kFineHalf ? cb - kFineHalf : 0;
    win_hi = win_lo + 2 * kFineHalf;
    if (gate_speculates(fin, gp.spec, gp.spos, ctl)) {
      const double t = __dmul_rn(pred, gp.spec_mult);
      tw = t > tw ? t : tw;
    }
  }
}

// Survivor test of a stored element under the filter decided after the gate
// that produced it (identity always survives; the threshold was applied when
// writing).
template <int NW>
__device__ inline bool survives(const Key<NW>& k, double c, const Filter& f, const uint8_t* pos,
                                int nbits) {
  if (!f.cap_active) return true;
  if (key_zero(k)) return true;
  const uint64_t b = abs_bits(c);
  if (b != f.kth_bits) return b > f.kth_bits;
  if (!f.tie_active) return true;
  Key<NW> ck = to_canonical(k, pos, nbits);
  Key<NW> tk;
#pragma unroll
  for (int i = 0; i < NW; ++i) tk.w[i] = f.tie_key[i];
  return canon_le(ck, tk);
}

// A class of the input as the concatenation of up to kMaxClasses regions.
struct ClassView {
  uint64_t base[kMaxClasses];
  uint64_t start[kMaxClasses + 1];
  int nseg;
  __device__ __forceinline__ uint64_t size() const { return start[nseg]; }
  __device__ __forceinline__ uint64_t phys(uint64_t i) const {
    int s = 0;
#pragma unroll
    for (int t = 1; t < kMaxClasses; ++t)
      if (t < nseg && i >= start[t]) s = t;
    return base[s] + (i - start[s]);
  }
};

__device__ inline ClassView make_view(const Plan* __restrict__ pp, int cls) {
  const Plan& p = *pp;
  ClassView v;
  const int nc = 1 << p.wc;
  v.nseg = nc;
  uint64_t acc = 0;
  for (int c = 0; c < kMaxClasses; ++c) {
    v.start[c] = acc;
    if (c < nc) {
      v.base[c] = p.base[c][cls];
      acc += p.cnt[c][cls];
    } else {
      v.base[c] = 0;
    }
  }
  v.start[kMaxClasses] = acc;
#pragma unroll
  for (int c = 1; c < kMaxClasses; ++c)
    if (c >= nc) v.start[c] = acc;
  return v;
}

// Pattern of the (x, z) bits of P on the support of Q (nb = 2 or 4 bits,
// rep positions one per byte of phpos): the index of the gate's tables.
template <int NW>
__device__ __forceinline__ uint32_t support_pattern(const Key<NW>& k, uint32_t phpos, uint32_t nb) {
  uint32_t idx = bit_at(k, phpos & 0xffu) | (bit_at(k, (phpos >> 8) & 0xffu) << 1);
  if (nb > 2) idx |= (bit_at(k, (phpos >> 16) & 0xffu) << 2) | (bit_at(k, phpos >> 24) << 3);
  return idx;
}

// e mod 4 of Q P = i^e R read from the gate's table over the support
// pattern of P (nph = 2 or 4 bits).
template <int NW>
__device__ __forceinline__ uint32_t phase_e(const Key<NW>& k, uint32_t phpos, uint32_t etab, uint32_t nph) {
  return (etab >> (2 * support_pattern(k, phpos, nph))) & 3u;
}

// Pauli weight (non-identity letters, Sec. II.B) of a key in a rep whose
// canonical bit b sits at rep position pos[b] (x bits of qubits 0..n-1,
// then their z bits).
template <int NW>
__device__ __forceinline__ uint32_t pauli_weight(const Key<NW>& k, const uint8_t* pos, int n) {
  uint32_t w = 0;
  for (int i = 0; i < n; ++i) w += bit_at(k, pos[i]) | bit_at(k, pos[n + i]);
  return w;
}

// Phase of Q P = sigma R for a commuting P: +1 or -1 (sigma_neg = 1 for -1).
// e = aQ + sum_j (xP zP - xR zR) + 2 sum_j zQ xP  (mod 4) over the support.
template <int NW>
__device__ __forceinline__ int phase_negative(const Key<NW>& k, const GateParams& gp) {
  int e = gp.aQ;
  for (int j = 0; j < gp.nsup; ++j) {
    const int xp = get_bit(k, gp.px[j]);
    const int zp = get_bit(k, gp.pz[j]);
    const int xr = xp ^ gp.qx[j];
    const int zr = zp ^ gp.qz[j];
    e += (xp & zp) - (xr & zr) + 2 * (gp.qz[j] & xp);
  }
  e &= 3;
  return e;  // 0: +1, 2: -1, odd: error
}

template <int NW>
__device__ __forceinline__ bool anticommutes(const Key<NW>& k, const GateParams& gp) {
  int par = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) par ^= __popcll(k.w[i] & gp.cmask[i]) & 1;
  return par != 0;
}

__device__ __forceinline__ uint32_t lane16(uint64_t v, int e) { return (uint32_t)((v >> (16 * e)) & 0xffffull); }

// ---------------------------------------------------------------------------
// Block-wide exclusive scan of two packed u64 vectors (16-bit lanes).
template <int BLOCK>
__device__ inline void block_scan2(uint64_t& a, uint64_t& b, uint64_t* wa, uint64_t* wb,
                                   uint64_t& tot_a, uint64_t& tot_b) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  constexpr int NWAVE = BLOCK / 64;
  uint64_t ia = a, ib = b;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint64_t ta = __shfl_up(ia, d, 64);
    uint64_t tb = __shfl_up(ib, d, 64);
    if (lane >= d) {
      ia += ta;
      ib += tb;
    }
  }
  if (lane == 63) {
    wa[wid] = ia;
    wb[wid] = ib;
  }
  __syncthreads();
  uint64_t pa = 0, pb = 0, sa = 0, sb = 0;
#pragma unroll
  for (int w = 0; w < NWAVE; ++w) {
    if (w < wid) {
      pa += wa[w];
      pb += wb[w];
    }
    sa += wa[w];
    sb += wb[w];
  }
  a = pa + ia - a;
  b = pb + ib - b;
  tot_a = sa;
  tot_b = sb;
  __syncthreads();
}

// End (exclusive) of output region (c, e) in the (c major, e minor) layout.
__device__ __forceinline__ uint64_t region_end(const uint64_t (*ob)[kMaxClasses], int c, int e) {
  int cc = c, ee = e + 1;
  if (ee == kMaxClasses) {
    ee = 0;
    ++cc;
  }
  return ob[cc][ee];
}

// Join layout shared by the partition and gate kernels: the classes of the
// gate's input, and for join j (classes j and ~j) its first tile and first
// boundary index.
struct JoinLayout {
  ClassView views[kMaxClasses];
  uint64_t tiles_before[kMaxClasses / 2 + 1];
  int njoin, full;
};

// Copy of a Plan in LDS made with one 4-byte load per thread (threads t in
// [0, sizeof(Plan)/4) take part; callers pass their thread index minus an
// offset to use other threads, and synchronise before reading).  The
// prologue arithmetic on a plan (class views, join layout, region bases) is
// a chain of dependent reads: from global memory, where the previous kernel
// left the plan, each would be a round trip of a microsecond or more.
__device__ __forceinline__ void plan_to_lds(Plan* dst, const Plan* __restrict__ src, int t) {
  static_assert(sizeof(Plan) % 4 == 0, "the plan is copied in 4-byte words");
  constexpr int kWords = (int)(sizeof(Plan) / 4);
  if (t >= 0 && t < kWords) reinterpret_cast<uint32_t*>(dst)[t] = reinterpret_cast<const uint32_t*>(src)[t];
}

__device__ inline void make_layout(JoinLayout& L, const Plan* __restrict__ pin, int w, int tile) {
  const int ncls = 1 << w;
  L.full = ncls - 1;
  L.njoin = ncls >> 1;
  for (int c = 0; c < kMaxClasses; ++c) L.views[c] = make_view(pin, c < ncls ? c : 0);
  L.tiles_before[0] = 0;
  for (int j = 0; j < kMaxClasses / 2; ++j) {
    uint64_t len = 0;
    if (j < L.njoin) len = L.views[j].size() + L.views[j ^ L.full].size();
    L.tiles_before[j + 1] = L.tiles_before[j] + (len + tile - 1) / tile;
  }
}


// Instantiations: key words (2: n <= 64, 4: n <= 128) x coefficient type.
#define ITPP_DISPATCH(nw, f32, KERNEL_CALL)            \
  do {                                                  \
    if (nw == 2 && !f32) {                              \
      constexpr int NWC = 2;                            \
      using TC = double;                                \
      KERNEL_CALL;                                      \
    } else if (nw == 2) {                               \
      constexpr int NWC = 2;                            \
      using TC = float;                                 \
      KERNEL_CALL;                                      \
    } else if (!f32) {                                  \
      constexpr int NWC = 4;                            \
      using TC = double;                                \
      KERNEL_CALL;                                      \
    } else {                                            \
      constexpr int NWC = 4;                            \
      using TC = float;                                 \
      KERNEL_CALL;                                      \
    }                                                   \
  } while (0)

}  // namespace itpp
