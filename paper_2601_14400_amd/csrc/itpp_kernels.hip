// HIP kernels of the ITPP layer update for gfx950 (wave64).
//
// One elementary gate exp(-(theta/2) Q) (Eq. ITPP_PropRules, Algorithm 1) is
// one pass of `gate_kernel` over the stored strings followed by the small
// selection kernels that decide the truncation (coefficient threshold of
// Sec. II.B and K-truncation of Sec. II.C) and the normalisation by the
// identity coefficient (Sec. II.C).  The truncation and normalisation are
// applied when the next gate loads its input ("deferred filter"), so every
// gate reads and writes the state exactly once.
//
// Pairing.  Keys are stored in a bit-permuted representation in which the
// bits flipped by the current gate are the most significant ones (see
// itpp_internal.h).  Strings with flip-bit pattern c ("class c") form a sorted
// sequence, and P -> Q P maps class c onto class ~c preserving order, so the
// partners of Eq. (ITPP_PropRules) are found by a merge-join of the two
// sorted sequences.  Merge-path tiles give every workgroup an equal share of
// the merged sequence; a pair straddling a tile boundary is moved into the
// earlier tile.  The merged output is written through a decoupled look-back
// prefix into regions sorted for the next gate (one LSD radix step fused
// into the write).
//
// Arithmetic (compiled with -ffp-contract=off): a commuting string with
// partner gives fl(fl(ch*c) + fl(-+sh*c')), without partner fl(ch*c) and a
// branch -+fl(sh*c); an anticommuting string keeps c.  Inputs are normalised
// on load with an IEEE division by the previous identity coefficient.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// ---------------------------------------------------------------------------
// Merge-path partition: eight tile boundaries per wavefront, each searched
// by a group of 8 lanes (8-ary search of the co-rank: the number of class-A
// strings among the first d of the merged sequence, A first on equal keys;
// few probes per level keep the scattered key reads small), then a pair
// split by the boundary is moved into the earlier tile.
template <int NW>
__global__ __launch_bounds__(256) void partition_kernel(GateParams gp, Side in, const Plan* __restrict__ plan_in,
                                                         uint64_t* __restrict__ part, Ctl* __restrict__ ctl) {
  __shared__ JoinLayout L;
  if (threadIdx.x == 0) make_layout(L, plan_in, gp.w, gp.tile);
  __syncthreads();
  if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kErrNone || ctl->halt) return;
  const int lane = threadIdx.x & 63;
  const int grp = lane >> 3, sl = lane & 7;
  const uint64_t b = ((uint64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * 8 + (uint64_t)grp;
  // boundary b -> join j, local boundary tl (join j owns tiles_before[j]+j .. tiles_before[j+1]+j)
  int j = -1;
  uint64_t tl = 0;
  for (int q = 0; q < L.njoin; ++q) {
    const uint64_t first = L.tiles_before[q] + q, last = L.tiles_before[q + 1] + q;
    if (b >= first && b <= last) {
      j = q;
      tl = b - first;
    }
  }
  bool valid = j >= 0;
  if (valid && b >= gp.status_cap + kMaxClasses) {
    if (sl == 0) atomicMax(&ctl->error, kErrCapacity);
    valid = false;
  }
  const int jj0 = valid ? j : 0;
  const ClassView& VA = L.views[jj0];
  const ClassView& VB = L.views[jj0 ^ L.full];
  const uint64_t nA = VA.size(), nB = VB.size(), len = nA + nB;
  const uint64_t d = (tl * (uint64_t)gp.tile < len) ? tl * (uint64_t)gp.tile : len;
  const int nbits = gp.nbits, w = gp.w;
  uint64_t lo = 0, hi = 0;  // answer in [lo, hi]
  if (valid) {
    lo = d > nB ? d - nB : 0;
    hi = d < nA ? d : nA;
  }
  // all groups of the wave step together until every search is done
  while (__ballot(hi > lo) != 0) {
    const bool active = hi > lo;
    const uint64_t range = hi - lo;
    const uint64_t step = active ? (range + 7) / 8 : 1;
    const uint64_t i = lo + (uint64_t)sl * step;
    bool pred = false;
    if (active && i < hi) {
      Key<NW> a = load_key<NW>(in, VA.phys(i));
      Key<NW> bb = xor_top(load_key<NW>(in, VB.phys(d - i - 1)), nbits, w);
      pred = !key_less(bb, a);  // A[i] <= B'[d-i-1]: the answer is above i
    }
    const uint64_t mask = __ballot(pred);
    if (active) {
      const int cnt = __popcll((mask >> (8 * grp)) & 0xffull);
      if (step == 1) {
        lo = lo + (uint64_t)cnt;
        hi = lo;
      } else {
        const uint64_t nlo = cnt == 0 ? lo : lo + (uint64_t)(cnt - 1) * step + 1;
        const uint64_t nhi_c = lo + (uint64_t)cnt * step;
        hi = nhi_c < hi ? nhi_c : hi;
        lo = nlo;
      }
    }
  }
  if (valid && sl == 0) {
    uint64_t i = lo, jj = d - lo;
    if (i > 0 && jj < nB) {
      Key<NW> a = load_key<NW>(in, VA.phys(i - 1));
      Key<NW> bb = xor_top(load_key<NW>(in, VB.phys(jj)), nbits, w);
      if (key_eq(a, bb)) jj += 1;
    }
    part[2 * b] = i;
    part[2 * b + 1] = jj;
  }
}

// ---------------------------------------------------------------------------
// The gate kernel: one merge-path tile per ticket (persistent workgroups).
//
// Per tile: (1) load the A range (class cA) and the B range (class cB, keys
// xored with the gate into cA's key space) with the previous gate's filter
// and normalisation applied; (2) every thread walks a contiguous run of the
// merged order (A before B on equal keys; an equal pair is one partner pair
// of Eq. ITPP_PropRules), computes the outputs and numbers them inside its
// run per output stream and next class; (3) a block scan turns run counts
// into tile ranks, a look-back across tiles of the same join turns them into
// region positions; (4) every element writes its outputs.
template <int NW, int BLOCK, int TILE, typename T>
struct GateSmem {
  static_assert(TILE + 1 < 4096, "tile counts are packed in 12-bit look-back fields");
  static constexpr int CAPT = TILE + 2;
  static constexpr int PER = (CAPT + BLOCK - 1) / BLOCK;
  uint64_t key[NW][CAPT];
  T coef[CAPT];
  uint16_t info[CAPT];  // bit0 survive, bit1 commuting, bit2 paired, bit3 self, bits4-5 its class,
                        // bit6 branch, bits7-8 its class
  uint16_t partner[CAPT];
  uint16_t rs[CAPT], rb[CAPT];  // ranks of the self / branch output inside the tile's stream and class
  uint64_t tot0, tot1;          // tile totals per next class (16-bit lanes): stream cA, stream cB
  uint64_t wa[BLOCK / 64], wb[BLOCK / 64];
  uint32_t fhist[kFineBins];
  uint32_t ncnt[kMaxClasses * kMaxClasses];
  uint64_t out_base[kMaxClasses + 1][kMaxClasses];  // row kMaxClasses holds the total
  uint32_t excl[2 * kMaxClasses];
  uint32_t tile;
  uint32_t nwritten, nabove;
  uint64_t pf[4];  // merge-path bounds of the tile: i0, j0, i1, j1
  JoinLayout L;
};

// Take the next tile ticket and read its merge-path bounds (one thread).
__device__ __forceinline__ void take_ticket(const JoinLayout& L, const uint64_t* __restrict__ part, Ctl* ctl,
                                            uint32_t& t, uint64_t pf[4]) {
  t = atomicAdd(&ctl->ticket, 1u);
  const uint64_t total = L.tiles_before[L.njoin];
  pf[0] = pf[1] = pf[2] = pf[3] = 0;
  if (t < total) {
    int j = 0;
    while (j + 1 < L.njoin && t >= L.tiles_before[j + 1]) ++j;
    const uint64_t pb = L.tiles_before[j] + (uint64_t)j + (t - L.tiles_before[j]);
#pragma unroll
    for (int q = 0; q < 4; ++q) pf[q] = part[2 * pb + q];
  }
}

__device__ __forceinline__ uint64_t phys_sel(const ClassView& v, uint64_t i) {
  uint64_t b = v.base[0], st = 0;
#pragma unroll
  for (int t = 1; t < kMaxClasses; ++t) {
    const bool in = (t < v.nseg) && (i >= v.start[t]);
    b = in ? v.base[t] : b;
    st = in ? v.start[t] : st;
  }
  return b + (i - st);
}

template <int NW, int TILE>
__device__ __forceinline__ Key<NW> lds_key(const uint64_t (*key)[TILE + 2], int x) {
  Key<NW> k;
#pragma unroll
  for (int q = 0; q < NW; ++q) k.w[q] = key[q][x];
  return k;
}

// New value of an element (Eq. ITPP_PropRules, then the branch of an
// unpaired commuting string); neg: Q P = -R.
template <typename T>
__device__ __forceinline__ void values_from(T c, bool comm, bool paired, T cp, bool neg, T ch, T sh, T& vs,
                                            T& vb) {
  vb = (T)0;
  if (!comm) {
    vs = c;
    return;
  }
  const T t1 = mul_rn(ch, c);
  if (paired) {
    T t2 = mul_rn(sh, cp);
    if (!neg) t2 = -t2;
    vs = add_rn(t1, t2);
  } else {
    vs = t1;
    T t2 = mul_rn(sh, c);
    if (!neg) t2 = -t2;
    vb = t2;
  }
}

// Reverse step (4) of one tile.  Element x survived the previous truncation
// (info bit 0), commutes with Q (bit 1), has a surviving partner (bit 2),
// and its self / branch output was written at a known position (bits 3 / 6).
// lambda_u at an output position is lambda'[pos] / b_I, minus s / b_I at the
// identity (the first element of the packed output), s = sum lambda' a'.
template <int NW, int BLOCK, int TILE, typename T, typename Smem>
__device__ void adjoint_tile(Smem& sm, const AdjArgs& adj, const GateParams& gp, const Filter& fin, T ch, T sh,
                             uint64_t t, int nAt, int nt, uint64_t i0, uint64_t j0, const ClassView& VA,
                             const ClassView& VB, int cA, int cB, Ctl* ctl) {
  const int tid = threadIdx.x;
  const double bI = adj.filt_next->cI;
  const double s_out = *adj.s_in;
  // pass 1: lambda_u at every element's self output, kept in the key array
  for (int x = tid; x < nt; x += BLOCK) {
    const uint16_t inf = sm.info[x];
    double lu = 0.0;
    if (inf & 8u) {
      const bool isA = x < nAt;
      const int es = (inf >> 4) & 3;
      const int cls = isA ? cA : cB;
      const uint64_t pos = sm.out_base[cls][es] + sm.excl[(isA ? 0 : 1) * kMaxClasses + es] + sm.rs[x];
      if (pos >= region_end(sm.out_base, cls, es)) {
        atomicMax(&ctl->error, kErrCapacity);
      } else {
        lu = adj.lam_out[pos] / bI;
        if (pos == 0) lu = lu - s_out / bI;
      }
    }
    sm.key[0][x] = (uint64_t)__double_as_longlong(lu);
  }
  __syncthreads();
  // pass 2: lambda at the inputs, dL/dtheta and sum lambda a
  double st = 0.0, ct = 0.0, ss = 0.0, cs = 0.0;
  for (int x = tid; x < nt; x += BLOCK) {
    const uint16_t inf = sm.info[x];
    const bool isA = x < nAt;
    const uint64_t p = isA ? phys_sel(VA, i0 + x) : phys_sel(VB, j0 + (x - nAt));
    double li = 0.0;
    if (inf & 1u) {
      const double a = (double)sm.coef[x];
      const double lu = __longlong_as_double((long long)sm.key[0][x]);
      if (!(inf & 2u)) {
        li = lu;
      } else {
        double lo = 0.0;
        if (inf & 4u) {
          lo = __longlong_as_double((long long)sm.key[0][sm.partner[x]]);
        } else if (inf & 64u) {
          const int eb = (inf >> 7) & 3;
          const int cls = isA ? cB : cA;
          const uint64_t pos = sm.out_base[cls][eb] + sm.excl[(isA ? 1 : 0) * kMaxClasses + eb] + sm.rb[x];
          if (pos >= region_end(sm.out_base, cls, eb)) {
            atomicMax(&ctl->error, kErrCapacity);
          } else {
            lo = adj.lam_out[pos] / bI;
            if (pos == 0) lo = lo - s_out / bI;
          }
        }
        const bool neg = (inf >> 9) & 1;  // Q P = -R
        const double chd = (double)ch, shd = (double)sh;
        const double t1 = __dmul_rn(chd, lu), t2 = __dmul_rn(shd, lo);
        li = neg ? __dadd_rn(t1, t2) : __dsub_rn(t1, t2);
        const double d1 = __dmul_rn(shd, lu), d2 = __dmul_rn(chd, lo);
        const double dt = __dmul_rn(a, neg ? __dadd_rn(d1, d2) : __dsub_rn(d1, d2));
        double sres, err;
        two_sum(st, dt, sres, err);
        st = sres;
        ct = __dadd_rn(ct, err);
      }
      double sres, err;
      two_sum(ss, __dmul_rn(li, a), sres, err);
      ss = sres;
      cs = __dadd_rn(cs, err);
    }
    adj.lam_in[p] = li;
  }
  // fixed-order block reduction of the two compensated sums (the key
  // arrays are free again and hold 4 * BLOCK doubles)
  static_assert(NW * (TILE + 2) >= 4 * BLOCK, "reduction scratch");
  double* red = reinterpret_cast<double*>(&sm.key[0][0]);
  __syncthreads();
  red[tid] = st;
  red[BLOCK + tid] = ct;
  red[2 * BLOCK + tid] = ss;
  red[3 * BLOCK + tid] = cs;
  __syncthreads();
  for (int h = BLOCK / 2; h > 0; h >>= 1) {
    if (tid < h) {
      double sres, err;
      two_sum(red[tid], red[tid + h], sres, err);
      red[tid] = sres;
      red[BLOCK + tid] = __dadd_rn(__dadd_rn(red[BLOCK + tid], red[BLOCK + tid + h]), err);
      two_sum(red[2 * BLOCK + tid], red[2 * BLOCK + tid + h], sres, err);
      red[2 * BLOCK + tid] = sres;
      red[3 * BLOCK + tid] = __dadd_rn(__dadd_rn(red[3 * BLOCK + tid], red[3 * BLOCK + tid + h]), err);
    }
    __syncthreads();
  }
  if (tid == 0) {
    adj.part[4 * t + 0] = red[0];
    adj.part[4 * t + 1] = red[BLOCK];
    adj.part[4 * t + 2] = red[2 * BLOCK];
    adj.part[4 * t + 3] = red[3 * BLOCK];
  }
  __syncthreads();
}

//
// ADJ = true is the reverse sweep of the same gate (frozen support): the
// load, walk, scan and look-back are those of the forward gate, so every
// element finds the positions its outputs had in the forward run's packed
// output; step (4) then gathers lambda' there and writes lambda for the input
// (adjoint of Eq. ITPP_PropRules, of the kept-set restriction and of the
// division by the identity coefficient), with per-tile partial sums of
// dL/dtheta and of sum lambda a.
template <int NW, int BLOCK, int TILE, typename T, bool ADJ>
__global__ __launch_bounds__(BLOCK, 4) void gate_kernel(GateParams gp, Side in, Side out,
                                                      const Plan* __restrict__ plan_in,
                                                      Plan* __restrict__ plan_out,
                                                      const Filter* __restrict__ filt_in,
                                                      const uint64_t* __restrict__ part,
                                                      Ctl* __restrict__ ctl,
                                                      TileStatus* __restrict__ status, AdjArgs adj) {
  using Smem = GateSmem<NW, BLOCK, TILE, T>;
  constexpr int PER = Smem::PER;
  __shared__ Smem sm;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // nothing at all (not even the plan prologue) after an error or a halt
  if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kErrNone || ctl->halt) return;
  const Filter fin = *filt_in;
  const T ch = (T)gp.ch, sh = (T)gp.sh;
  const int nbits = gp.nbits;
  const int w = gp.w;
  const int ncls = 1 << w;
  const int full = ncls - 1;
  const int ncls1 = 1 << gp.w1;
  // fine histogram window around the value predicted from the previous cap
  uint64_t win_lo = 0, win_hi = 0;
  double tw = gp.delta;  // outputs are written when |v| > tw
  if (fin.ref_bits) {
    const double pred = __longlong_as_double((long long)fin.ref_bits) / fin.cI;
    const uint64_t cb = abs_bits(pred);
    win_lo = cb > kFineHalf ? cb - kFineHalf : 0;
    win_hi = win_lo + 2 * kFineHalf;
    if (gp.spec && fin.cap_active) {
      const double t = __dmul_rn(pred, gp.spec_mult);
      tw = t > tw ? t : tw;
    }
  }

  for (int i = tid; i < kFineBins; i += BLOCK) sm.fhist[i] = 0;
  if (tid < kMaxClasses * kMaxClasses) sm.ncnt[tid] = 0;
  if (tid == 0) {
    const Plan* __restrict__ pin = plan_in;
    uint64_t acc = 0;
    if constexpr (ADJ) {
      // the forward output, packed: region (c, e) holds exactly cnt[c][e]
      const Plan* __restrict__ pn = adj.plan_next;
      for (int c = 0; c < kMaxClasses; ++c)
        for (int e = 0; e < kMaxClasses; ++e) {
          sm.out_base[c][e] = acc;
          if (c < ncls && e < ncls1) acc += pn->cnt[c][e];
        }
      if (pn->base[0][0] != 0 || acc > adj.lam_out_len) atomicMax(&ctl->error, kErrCapacity);
      if (blockIdx.x == 0) *adj.ntiles = 0;
    } else {
      // output region capacities: cap(c,e) = n[c][e] + n[~c][e ^ ov]
      for (int c = 0; c < kMaxClasses; ++c)
        for (int e = 0; e < kMaxClasses; ++e) {
          sm.out_base[c][e] = acc;
          if (c < ncls && e < ncls1) acc += (uint64_t)pin->ncnt[c][e] + (uint64_t)pin->ncnt[c ^ full][e ^ gp.ov];
        }
    }
    for (int e = 0; e < kMaxClasses; ++e) sm.out_base[kMaxClasses][e] = acc;
    if (acc > gp.cap_elems) atomicMax(&ctl->error, kErrCapacity);
    if (blockIdx.x == 0 && !ADJ) {
      for (int c = 0; c < kMaxClasses; ++c)
        for (int e = 0; e < kMaxClasses; ++e) plan_out->base[c][e] = sm.out_base[c][e];
      plan_out->wc = w;
      plan_out->we = gp.w1;
    }
    sm.nwritten = 0;
    sm.nabove = 0;
    make_layout(sm.L, pin, w, TILE);
  }
  __syncthreads();
  const uint64_t total_tiles = sm.L.tiles_before[sm.L.njoin];
  if constexpr (ADJ) {
    if (blockIdx.x == 0 && tid == 0) *adj.ntiles = total_tiles;
  }
  if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kErrNone || ctl->halt) return;
  if (tid == 0) {
    uint32_t t0;
    uint64_t pf[4];
    take_ticket(sm.L, part, ctl, t0, pf);
    sm.tile = t0;
#pragma unroll
    for (int q = 0; q < 4; ++q) sm.pf[q] = pf[q];
  }
  __syncthreads();

  for (;;) {
    const uint64_t t = sm.tile;
    if (t >= total_tiles) break;
    if (t >= gp.status_cap) {
      if (tid == 0) atomicMax(&ctl->error, kErrCapacity);
      break;
    }
    int j = 0;
    while (j + 1 < sm.L.njoin && t >= sm.L.tiles_before[j + 1]) ++j;
    const uint64_t tl = t - sm.L.tiles_before[j];
    const int cA = j, cB = j ^ full;
    const ClassView VA = sm.L.views[cA];
    const ClassView VB = sm.L.views[cB];
    (void)tl;
    const uint64_t i0 = sm.pf[0], j0 = sm.pf[1];
    const int nAt = (int)(sm.pf[2] - i0);
    const int nBt = (int)(sm.pf[3] - j0);
    const int nt = nAt + nBt;
    if (nt > TILE + 1 || nAt < 0 || nBt < 0) {
      if (tid == 0) atomicMax(&ctl->error, kErrCapacity);
      break;
    }

    // (1) load, filter, normalise
    for (int x = tid; x < nt; x += BLOCK) {
      const bool isA = x < nAt;
      const uint64_t p = isA ? phys_sel(VA, i0 + x) : phys_sel(VB, j0 + (x - nAt));
      Key<NW> k = load_key<NW>(in, p);
      const T cs = coefs<T>(in)[p];
      const bool sv = survives(k, (double)cs, fin, gp.pos_in, nbits);
      const bool comm = !anticommutes(k, gp);
      if (!isA) k = xor_top(k, nbits, w);  // B' = B xor Q lives in class cA's key space
#pragma unroll
      for (int q = 0; q < NW; ++q) sm.key[q][x] = k.w[q];
      sm.coef[x] = normalised<T>(cs, fin.cI);
      sm.info[x] = (uint16_t)((sv ? 1 : 0) | (comm ? 2 : 0));
    }
    __syncthreads();

    // (2) merge walk over merged positions [m0, m0 + PER): one element per
    // step, A before B on equal keys; an equal B follows its A partner
    uint64_t c0 = 0, c1 = 0;  // run counts per next class (16-bit lanes): stream cA, stream cB
    int xs[PER];              // element handled at step s
#pragma unroll
    for (int q = 0; q < PER; ++q) xs[q] = -1;
    {
      const int m0 = tid * PER;
      const int m1 = (m0 + PER < nt) ? m0 + PER : nt;
      if (m0 < nt) {
        int lo = m0 > nBt ? m0 - nBt : 0;
        int hi = m0 < nAt ? m0 : nAt;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          const Key<NW> ka = lds_key<NW, TILE>(sm.key, mid);
          const Key<NW> kb = lds_key<NW, TILE>(sm.key, nAt + (m0 - mid - 1));
          if (!key_less(kb, ka))
            lo = mid + 1;
          else
            hi = mid;
        }
        int a = lo, b = m0 - lo;
#pragma unroll
        for (int step = 0; step < PER; ++step) {
          if (a + b >= m1) break;
          const bool haveA = a < nAt, haveB = b < nBt;
          Key<NW> ka, kb;
          if (haveA) ka = lds_key<NW, TILE>(sm.key, a);
          if (haveB) kb = lds_key<NW, TILE>(sm.key, nAt + b);
          const bool isA = haveA && (!haveB || !key_less(kb, ka));
          const int x = isA ? a : nAt + b;
          // partner: for A the current B if equal, for B the previous A if equal
          int y = -1;
          if (isA) {
            if (haveB && key_eq(ka, kb)) y = nAt + b;
          } else if (a > 0) {
            if (key_eq(lds_key<NW, TILE>(sm.key, a - 1), kb)) y = a - 1;
          }
          const Key<NW> k = isA ? ka : kb;
          uint16_t inf = sm.info[x];
          const bool sv = inf & 1, comm = (inf >> 1) & 1;
          uint16_t rsx = 0, rbx = 0;
          if (sv) {
            const bool paired = (y >= 0) && (sm.info[y] & 1);
            const T c = sm.coef[x];
            const T cp = paired ? sm.coef[y] : (T)0;
            const Key<NW> ownk = isA ? k : xor_top(k, nbits, w);
            bool neg = false;
            if (comm) {
              const int e4 = phase_negative(ownk, gp);
              if (e4 & 1) atomicMax(&ctl->error, kErrPhase);
              neg = (e4 == 2);
              if (neg) inf |= 512u;
            }
            T vs, vb;
            values_from<T>(c, comm, paired, cp, neg, ch, sh, vs, vb);
            const bool hs = abs_d(vs) > tw;
            const bool hb = comm && !paired && abs_d(vb) > tw;
            if (paired) {
              inf |= 4u;
              sm.partner[x] = (uint16_t)y;
            }
            int es = 0;
            for (int mm = 0; mm < gp.w1; ++mm) es |= get_bit(ownk, gp.epos[mm]) << mm;
            // A: self -> stream cA, branch -> stream cB; B: the reverse
            uint64_t sinc = 0, binc = 0;
            if (hs) {
              inf |= (uint16_t)(8u | (es << 4));
              sinc = 1ull << (16 * es);
              rsx = (uint16_t)lane16(isA ? c0 : c1, es);
            }
            if (hb) {
              const int eb = es ^ gp.ov;  // the branch differs in this gate's bits only
              inf |= (uint16_t)(64u | (eb << 7));
              binc = 1ull << (16 * eb);
              rbx = (uint16_t)lane16(isA ? c1 : c0, eb);
            }
            c0 += isA ? sinc : binc;
            c1 += isA ? binc : sinc;
          }
          sm.info[x] = inf;
          sm.rs[x] = rsx;
          sm.rb[x] = rbx;
          xs[step] = x;
          if (isA) ++a;
          else ++b;
        }
      }
    }
    // (3) block scan of the run counts; ranks of this thread's outputs become tile ranks
    {
      uint64_t t0, t1;
      uint64_t p0 = c0, p1 = c1;
      block_scan2<BLOCK>(p0, p1, sm.wa, sm.wb, t0, t1);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int x = xs[q];
        if (x < 0) continue;
        const uint16_t inf = sm.info[x];
        const bool isA = x < nAt;
        if (inf & 8u) sm.rs[x] = (uint16_t)(sm.rs[x] + lane16(isA ? p0 : p1, (inf >> 4) & 3));
        if (inf & 64u) sm.rb[x] = (uint16_t)(sm.rb[x] + lane16(isA ? p1 : p0, (inf >> 7) & 3));
      }
      if (tid == 0) {
        sm.tot0 = t0;
        sm.tot1 = t1;
      }
    }
    __syncthreads();
    // look-back across the tiles of this join (wave 0)
    if (tid < 64) {
      uint32_t agg[2 * kMaxClasses];
#pragma unroll
      for (int e = 0; e < kMaxClasses; ++e) {
        agg[e] = lane16(sm.tot0, e);
        agg[kMaxClasses + e] = lane16(sm.tot1, e);
      }
      constexpr int NQ = 2 * kMaxClasses;
      const uint64_t SN = gp.status_cap;
      const unsigned long long tag32 = (unsigned long long)gp.epoch << 32;
      const unsigned long long tag12 = (unsigned long long)(gp.epoch % 4095u + 1u) << 52;
      const unsigned long long kInclReady = 1ull << 48;
      unsigned long long aw[2];
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        unsigned long long v = tag12;
#pragma unroll
        for (int e = 0; e < kMaxClasses; ++e) v |= (unsigned long long)agg[sd * kMaxClasses + e] << (12 * e);
        aw[sd] = v;
      }
      uint32_t excl[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) excl[q] = 0;
      if (tl == 0) {
        if (lane == 0) {
#pragma unroll
          for (int q = 0; q < NQ; ++q)
            __hip_atomic_store(&status[(2 + q) * SN + t], tag32 | agg[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
          for (int sd = 0; sd < 2; ++sd)
            __hip_atomic_store(&status[sd * SN + t], aw[sd] | kInclReady, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      } else {
        if (lane == 0) {
#pragma unroll
          for (int sd = 0; sd < 2; ++sd)
            __hip_atomic_store(&status[sd * SN + t], aw[sd], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // each lane inspects LB consecutive predecessors per round (window 64 * LB)
        constexpr int LB = 2;
        const int64_t first = (int64_t)sm.L.tiles_before[j];
        int64_t khi = (int64_t)t - 1;
        bool done = false;
        while (!done) {
          unsigned long long w0[LB], w1[LB];
          // position r*64 + lane is predecessor khi - (r*64 + lane): one
          // coalesced load of 64 consecutive tiles per r.  All rows are in
          // flight together; rows whose record carries an older epoch are
          // read again until the predecessor has published.
          uint32_t pend = 0;
#pragma unroll
          for (int r = 0; r < LB; ++r) {
            w0[r] = kInclReady;  // before the join's first tile: never needed, reads as ready with zero
            w1[r] = 0;
            if (khi - (int64_t)(r * 64 + lane) >= first) pend |= 1u << r;
          }
          uint32_t spins = 0;
          while (pend) {
#pragma unroll
            for (int r = 0; r < LB; ++r) {
              if ((pend >> r) & 1u) {
                const int64_t k = khi - (int64_t)(r * 64 + lane);
                w0[r] = __hip_atomic_load(&status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                w1[r] = __hip_atomic_load(&status[SN + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              }
            }
#pragma unroll
            for (int r = 0; r < LB; ++r)
              if (((pend >> r) & 1u) && (w0[r] >> 52) == (tag12 >> 52) && (w1[r] >> 52) == (tag12 >> 52))
                pend &= ~(1u << r);
            if (!pend) break;
            if (++spins > (1u << 22)) {
              atomicMax(&ctl->error, kErrSpin);
#pragma unroll
              for (int r = 0; r < LB; ++r)
                if ((pend >> r) & 1u) {
                  w0[r] = kInclReady;
                  w1[r] = 0;
                }
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          // nearest predecessor whose inclusive prefix is published
          uint32_t best = 64 * LB;
#pragma unroll
          for (int r = LB - 1; r >= 0; --r)
            if (w0[r] & kInclReady) best = (uint32_t)(r * 64 + lane);
#pragma unroll
          for (int d = 32; d >= 1; d >>= 1) {
            const uint32_t o = __shfl_xor(best, d, 64);
            best = o < best ? o : best;
          }
          // aggregates of the predecessors nearer than that one
          uint32_t sum[NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) sum[q] = 0;
#pragma unroll
          for (int r = 0; r < LB; ++r) {
            if ((uint32_t)(r * 64 + lane) < best) {
#pragma unroll
              for (int e = 0; e < kMaxClasses; ++e) {
                sum[e] += (uint32_t)((w0[r] >> (12 * e)) & 0xfffull);
                sum[kMaxClasses + e] += (uint32_t)((w1[r] >> (12 * e)) & 0xfffull);
              }
            }
          }
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            uint32_t v = sum[q];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
            excl[q] += v;
          }
          done = best < (uint32_t)(64 * LB);
          if (done) {
            const int64_t kp = khi - (int64_t)best;
            if (kp >= first) {
              // inclusive prefix of that predecessor (lane q reads counter q)
              uint32_t iv = 0;
              if (lane < NQ) {
                uint32_t spins = 0;
                for (;;) {
                  const unsigned long long x =
                      __hip_atomic_load(&status[(2 + lane) * SN + kp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                  if ((x >> 32) == gp.epoch) {
                    iv = (uint32_t)x;
                    break;
                  }
                  if (++spins > (1u << 22)) {
                    atomicMax(&ctl->error, kErrSpin);
                    break;
                  }
                  __builtin_amdgcn_s_sleep(1);
                }
              }
#pragma unroll
              for (int q = 0; q < NQ; ++q) excl[q] += __shfl(iv, q, 64);
            }
          }
          khi -= 64 * LB;
        }
        if (lane == 0) {
#pragma unroll
          for (int q = 0; q < NQ; ++q)
            __hip_atomic_store(&status[(2 + q) * SN + t], tag32 | (excl[q] + agg[q]), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
          __atomic_thread_fence(__ATOMIC_RELEASE);
#pragma unroll
          for (int sd = 0; sd < 2; ++sd)
            __hip_atomic_store(&status[sd * SN + t], aw[sd] | kInclReady, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
      if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 2 * kMaxClasses; ++q) sm.excl[q] = excl[q];
        // the last tile of the join publishes the region fill counts
        if (!ADJ && t + 1 == sm.L.tiles_before[j + 1]) {
#pragma unroll
          for (int e = 0; e < kMaxClasses; ++e) {
            if (e < ncls1) {
              plan_out->cnt[cA][e] = excl[e] + agg[e];
              plan_out->cnt[cB][e] = excl[kMaxClasses + e] + agg[kMaxClasses + e];
            }
          }
        }
      }
    }
    if constexpr (!ADJ) {
      // while wave 0 looks back, the other waves move the keys of the
      // elements with outputs into the next rep (one bit move per element)
      // and note the flip pattern of the gate after next (info bits 10-11)
      for (int x = tid; x < nt; x += BLOCK) {
        const uint16_t inf = sm.info[x];
        if (!(inf & (8u | 64u))) continue;
        const Key<NW> k = lds_key<NW, TILE>(sm.key, x);
        Key<NW> mk = k;
        for (int mm = 0; mm < gp.w1; ++mm) mk = move_top(mk, gp.mv[mm], nbits);
        const Key<NW> ownk = x < nAt ? k : xor_top(k, nbits, w);
        int fself = 0;
        for (int bq = 0; bq < gp.w2; ++bq) fself |= get_bit(ownk, gp.fposg[bq]) << bq;
#pragma unroll
        for (int q = 0; q < NW; ++q) sm.key[q][x] = mk.w[q];
        sm.info[x] = (uint16_t)(inf | (fself << 10));
      }
    }
    __syncthreads();
    if constexpr (ADJ) {
      adjoint_tile<NW, BLOCK, TILE, T>(sm, adj, gp, fin, ch, sh, t, nAt, nt, i0, j0, VA, VB, cA, cB, ctl);
      if (tid == 0) {
        uint32_t tn;
        uint64_t pf[4];
        take_ticket(sm.L, part, ctl, tn, pf);
        sm.tile = tn;
#pragma unroll
        for (int q = 0; q < 4; ++q) sm.pf[q] = pf[q];
      }
      __syncthreads();
      continue;
    }
    // (4) write outputs
    uint32_t written = 0, above = 0;
    for (int x = tid; x < nt; x += BLOCK) {
      const uint16_t inf = sm.info[x];
      if (!(inf & (8u | 64u))) continue;
      const bool isA = x < nAt;
      const bool paired = (inf >> 2) & 1;
      T vs, vb;
      values_from<T>(sm.coef[x], (inf >> 1) & 1, paired, paired ? sm.coef[sm.partner[x]] : (T)0, (inf >> 9) & 1,
                     ch, sh, vs, vb);
      // next-rep keys: the two outputs differ by this gate's mask
      const Key<NW> mk = lds_key<NW, TILE>(sm.key, x);
      Key<NW> mq = mk;
#pragma unroll
      for (int q = 0; q < NW; ++q) mq.w[q] ^= gp.qm1[q];
      const int fself = (inf >> 10) & 3;
      if (inf & 8u) {
        const int es = (inf >> 4) & 3;
        const int stream = isA ? 0 : 1;
        const int cls = isA ? cA : cB;
        const uint64_t pos = sm.out_base[cls][es] + sm.excl[stream * kMaxClasses + es] + sm.rs[x];
        const Key<NW>& ks = isA ? mk : mq;
        if (pos >= region_end(sm.out_base, cls, es)) {
          atomicMax(&ctl->error, kErrCapacity);
        } else {
          store_key<NW>(out, pos, ks);
          coefs<T>(out)[pos] = vs;
          if (key_zero(ks)) {
            ctl->cI_out = (double)vs;
            ctl->have_cI = 1u;
          } else {
            const uint64_t bits = abs_bits((double)vs);
            if (bits >= win_hi) ++above;
            else if (bits >= win_lo) atomicAdd(&sm.fhist[(bits - win_lo) >> kFineShift], 1u);
            ++written;
          }
          atomicAdd(&sm.ncnt[es * kMaxClasses + fself], 1u);
        }
      }
      if (inf & 64u) {
        const int eb = (inf >> 7) & 3;
        const int stream = isA ? 1 : 0;
        const int cls = isA ? cB : cA;
        const uint64_t pos = sm.out_base[cls][eb] + sm.excl[stream * kMaxClasses + eb] + sm.rb[x];
        const Key<NW>& kb = isA ? mq : mk;
        if (pos >= region_end(sm.out_base, cls, eb)) {
          atomicMax(&ctl->error, kErrCapacity);
        } else {
          store_key<NW>(out, pos, kb);
          coefs<T>(out)[pos] = vb;
          const uint64_t bits = abs_bits((double)vb);
          if (bits >= win_hi) ++above;
          else if (bits >= win_lo) atomicAdd(&sm.fhist[(bits - win_lo) >> kFineShift], 1u);
          ++written;
          atomicAdd(&sm.ncnt[eb * kMaxClasses + (fself ^ gp.ovf)], 1u);
        }
      }
    }
    if (written) atomicAdd(&sm.nwritten, written);
    if (above) atomicAdd(&sm.nabove, above);
    // the next ticket is taken only once this tile's work is done, so tiles
    // start in ticket order (the look-back relies on it); t and the bounds
    // were read into registers at the top of this tile
    if (tid == BLOCK - 1) {
      uint32_t tn;
      uint64_t pf[4];
      take_ticket(sm.L, part, ctl, tn, pf);
      sm.tile = tn;
#pragma unroll
      for (int q = 0; q < 4; ++q) sm.pf[q] = pf[q];
    }
    __syncthreads();
  }
  // flush per-workgroup statistics
  __syncthreads();
  if constexpr (ADJ) return;
  if (win_hi > win_lo)
    for (int i = tid; i < kFineBins; i += BLOCK) {
      const uint32_t v = sm.fhist[i];
      if (v) atomicAdd(&ctl->fhist[i], v);
    }
  if (tid < kMaxClasses * kMaxClasses) {
    const uint32_t v = sm.ncnt[tid];
    if (v) atomicAdd(&plan_out->ncnt[tid / kMaxClasses][tid % kMaxClasses], v);
  }
  if (tid == 0) {
    if (sm.nwritten) atomicAdd((unsigned long long*)&ctl->n_written_nonid, (unsigned long long)sm.nwritten);
    if (sm.nabove) atomicAdd((unsigned long long*)&ctl->n_above_hi, (unsigned long long)sm.nabove);
  }
}

// ---------------------------------------------------------------------------
// rho = I: one identity string with coefficient 1 (Algorithm 1 initial state).
template <int NW, typename T>
__global__ void init_kernel(Side s0, Plan* plan, Filter* filt, Ctl* ctl, int w0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < NW; ++q) s0.kw[q][0] = 0ull;
  coefs<T>(s0)[0] = (T)1;
  Plan p = {};
  p.cnt[0][0] = 1;
  p.ncnt[0][0] = 1;
  p.wc = 0;
  p.we = w0;
  plan[0] = p;
  Plan z = {};
  plan[1] = z;
  Filter f = {};
  f.cI = 1.0;
  f.n_written = 1;
  f.n_survivors = 1;
  *filt = f;
  Ctl c = {};
  *ctl = c;
}

// Parallel search, over a histogram of 2 * blockDim bins taken from the top,
// for the bin where the running count from above first reaches `need`
// (counts above the histogram: `base`).  Returns the bin (or -1) and the
// count above it; all threads must call.
__device__ inline void find_from_top(const uint32_t* h, int nbins, uint64_t base, uint64_t need,
                                     uint64_t* s_scratch, int* out_bin, uint64_t* out_above) {
  const int tid = threadIdx.x;
  const int nth = blockDim.x;
  const int per = (nbins + nth - 1) / nth;
  // thread t owns bins nbins-1-t*per .. nbins-per-t*per (descending)
  uint64_t local = 0;
  for (int q = 0; q < per; ++q) {
    const int b = nbins - 1 - (tid * per + q);
    if (b >= 0) local += h[b];
  }
  s_scratch[tid] = local;
  __syncthreads();
  // Hillis-Steele inclusive scan over threads (nth <= 1024)
  for (int d = 1; d < nth; d <<= 1) {
    const uint64_t v = (tid >= d) ? s_scratch[tid - d] : 0;
    __syncthreads();
    s_scratch[tid] += v;
    __syncthreads();
  }
  uint64_t above = base + s_scratch[tid] - local;
  for (int q = 0; q < per; ++q) {
    const int b = nbins - 1 - (tid * per + q);
    if (b < 0) break;
    if (above < need && need <= above + h[b]) {
      *out_bin = b;
      *out_above = above;
    }
    above += h[b];
  }
  __syncthreads();
}

// After a gate: check the identity coefficient, decide whether the cap
// binds and which bit range of |c| holds the (K-1)-th largest non-identity
// value; prepare the control block for the next gate.
__global__ __launch_bounds__(1024) void select_decide(const Filter* filt_in, Filter* filt_out, Plan* plan_next,
                                                      Ctl* ctl, int64_t K, int cap_fail, int spec,
                                                      uint64_t serial) {
  __shared__ uint32_t fh[kFineBins];
  __shared__ uint64_t scr[1024];
  __shared__ int s_bin;
  __shared__ uint64_t s_above;
  const int tid = threadIdx.x;
  if (ctl->error || ctl->halt) return;
  {
    // a speculative gate that wrote fewer than K-1 strings above its write
    // threshold cannot decide the cap exactly: ask the host to redo it
    const Filter& f0 = *filt_in;
    if (spec && f0.cap_active && (int64_t)ctl->n_written_nonid < K - 1) {
      __syncthreads();
      if (tid == 0) {
        ctl->halt = 1u;
        ctl->halt_serial = serial;
      }
      return;
    }
  }
  for (int i = tid; i < kFineBins; i += blockDim.x) fh[i] = ctl->fhist[i];
  if (tid == 0) {
    s_bin = -1;
    s_above = 0;
  }
  __syncthreads();
  const Filter fin = *filt_in;
  const uint64_t nw = ctl->n_written_nonid + 1;  // identity included
  const bool capped = (int64_t)nw > K;
  const uint64_t need = (uint64_t)(K - 1);
  uint64_t sel_lo = 0, sel_hi = 0, sel_need = 0;
  bool none_kept = false, coarse = false;
  if (capped && need == 0) {
    none_kept = true;
  } else if (capped) {
    uint64_t win_lo = 0, win_hi = 0;
    if (fin.ref_bits) {
      const double pred = __longlong_as_double((long long)fin.ref_bits) / fin.cI;
      const uint64_t cb = abs_bits(pred);
      win_lo = cb > kFineHalf ? cb - kFineHalf : 0;
      win_hi = win_lo + 2 * kFineHalf;
    }
    const uint64_t nab = ctl->n_above_hi;
    bool fine_ok = false;
    if (win_hi > win_lo && nab < need) {
      find_from_top(fh, kFineBins, nab, need, scr, &s_bin, &s_above);
      if (s_bin >= 0) {
        fine_ok = true;
        sel_lo = win_lo + ((uint64_t)s_bin << kFineShift);
        sel_hi = sel_lo + (1ull << kFineShift);
        sel_need = need - s_above;
      }
      __syncthreads();
      if (tid == 0) s_bin = -1;
      __syncthreads();
    }
    coarse = !fine_ok;
  }
  __syncthreads();
  for (int i = tid; i < kFineBins; i += blockDim.x) ctl->fhist[i] = 0;
  if (tid < kMaxClasses * kMaxClasses) {
    plan_next->cnt[tid / kMaxClasses][tid % kMaxClasses] = 0;
    plan_next->ncnt[tid / kMaxClasses][tid % kMaxClasses] = 0;
  }
  if (tid == 0) {
    const double cI = ctl->cI_out;
    uint32_t err = 0;
    if (!ctl->have_cI || !(cI > 0.0) || !isfinite(cI)) err = kErrNumeric;
    if (capped && cap_fail) err = kErrCap;
    if (err) atomicMax(&ctl->error, err);
    Filter f = {};
    f.cI = ctl->have_cI ? cI : 1.0;
    f.n_written = nw;
    f.cap_active = capped ? 1u : 0u;
    f.kth_bits = none_kept ? 0x7fffffffffffffffull : 0ull;
    f.tie_active = 0;
    f.n_survivors = capped ? (uint64_t)K : nw;
    // reference for the next gate's window: the exact K-th value once known
    // (select_exact), else the previous reference carried into this scale
    f.ref_bits = 0;
    if (!capped && fin.ref_bits) f.ref_bits = abs_bits(__longlong_as_double((long long)fin.ref_bits) / fin.cI);
    *filt_out = f;
    ctl->term_updates += (double)fin.n_survivors;
    ctl->alg_elems += (double)fin.n_survivors + (double)f.n_survivors;
    ctl->gates += 1;
    if (spec && fin.cap_active) ctl->spec_gates += 1;
    if (capped) ctl->cap_hit = 1;
    ctl->sel_lo = sel_lo;
    ctl->sel_hi = sel_hi;
    ctl->sel_need = (capped && !none_kept) ? (uint32_t)sel_need : 0u;
    ctl->need_coarse = (capped && !none_kept && coarse) ? 1u : 0u;
    if (ctl->need_coarse) ctl->sel_need = (uint32_t)need;  // resolved by select_coarse_hist
    ctl->cand_count = 0;
    ctl->ticket = 0;
    ctl->n_written_nonid = 0;
    ctl->n_above_hi = 0;
    ctl->have_cI = 0;
  }
}

// Reset the look-back records (their 12-bit epoch tags repeat every 4095
// gates; the host clears them more often than that).
__global__ void clear_status_kernel(TileStatus* status, uint64_t n) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n; i += stride) status[i] = 0;
}

hipError_t launch_clear_status(TileStatus* status, uint64_t n, hipStream_t st) {
  hipLaunchKernelGGL(clear_status_kernel, dim3(256), dim3(256), 0, st, status, n);
  return hipGetLastError();
}

// Clear what a gate accumulates, before a gate is redone after a failed
// speculation (select_decide does this for the following gate otherwise).
__global__ void prepare_kernel(Plan* plan_out, Ctl* ctl) {
  const int tid = threadIdx.x;
  for (int i = tid; i < kHistBins; i += blockDim.x) ctl->hist[i] = 0;
  for (int i = tid; i < kFineBins; i += blockDim.x) ctl->fhist[i] = 0;
  if (tid < kMaxClasses * kMaxClasses) {
    plan_out->cnt[tid / kMaxClasses][tid % kMaxClasses] = 0;
    plan_out->ncnt[tid / kMaxClasses][tid % kMaxClasses] = 0;
  }
  if (tid == 0) {
    ctl->ticket = 0;
    ctl->n_written_nonid = 0;
    ctl->n_above_hi = 0;
    ctl->have_cI = 0;
    ctl->cand_count = 0;
    ctl->sel_need = 0;
    ctl->need_coarse = 0;
    ctl->halt = 0;
  }
}

// Fallback when the K-th value is outside the fine window: full histogram of
// the stored non-identity |c| values (16 bins per octave); the last
// workgroup to finish picks the bin that holds the (K-1)-th value.
template <int NW, typename T>
__global__ __launch_bounds__(256) void select_coarse_hist(Side out, const Plan* plan, Ctl* ctl) {
  __shared__ uint32_t h[kHistBins];
  __shared__ uint64_t scr[256];
  __shared__ int s_bin;
  __shared__ uint64_t s_above;
  __shared__ uint32_t s_last;
  if (ctl->error || ctl->halt || !ctl->need_coarse) return;
  const int tid = threadIdx.x;
  for (int i = tid; i < kHistBins; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const Plan& p = *plan;
  const int nc = 1 << p.wc, ne = 1 << p.we;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (int c = 0; c < nc; ++c)
    for (int e = 0; e < ne; ++e) {
      const uint64_t base = p.base[c][e];
      const uint64_t cnt = p.cnt[c][e];
      for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + tid; i < cnt; i += stride) {
        if (c == 0 && e == 0 && i == 0) continue;  // the identity is the first string of region (0,0)
        atomicAdd(&h[hist_bin(abs_bits((double)coefs<T>(out)[base + i]))], 1u);
      }
    }
  __syncthreads();
  for (int i = tid; i < kHistBins; i += blockDim.x)
    if (h[i]) atomicAdd(&ctl->hist[i], h[i]);
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(&ctl->hist_done, 1u) == gridDim.x - 1 ? 1u : 0u;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  for (int i = tid; i < kHistBins; i += blockDim.x)
    h[i] = __hip_atomic_load(&ctl->hist[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (tid == 0) {
    s_bin = -1;
    s_above = 0;
  }
  __syncthreads();
  const uint64_t need = ctl->sel_need;
  find_from_top(h, kHistBins, 0, need, scr, &s_bin, &s_above);
  const int bsel = s_bin < 0 ? 0 : s_bin;
  for (int i = tid; i < kHistBins; i += blockDim.x) ctl->hist[i] = 0;
  if (tid == 0) {
    ctl->sel_lo = bsel == 0 ? 0ull : ((uint64_t)(bsel + kHistBase) << kHistShift);
    ctl->sel_hi = bsel == kHistBins - 1 ? ~0ull : ((uint64_t)(bsel + 1 + kHistBase) << kHistShift);
    ctl->sel_need = (uint32_t)(need - (s_bin < 0 ? 0 : s_above));
    ctl->need_coarse = 0;
    ctl->hist_done = 0;
  }
}

// Collect the stored non-identity elements whose |c| bits lie in the
// selected range.
template <int NW, typename T>
__global__ void select_collect(Side out, const Plan* plan, Ctl* ctl, SelBuf sel) {
  if (ctl->error || ctl->halt || ctl->sel_need == 0) return;
  const uint64_t lo = ctl->sel_lo, hi = ctl->sel_hi;
  const Plan& p = *plan;
  const int nc = 1 << p.wc, ne = 1 << p.we;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;  // a multiple of 64
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < nc; ++c)
    for (int e = 0; e < ne; ++e) {
      const uint64_t base = p.base[c][e];
      const uint64_t cnt = p.cnt[c][e];
      // wave-uniform loop over four strided chunks of 64 (their loads are
      // in flight together); one atomic per wave reserves the wave's slots
      constexpr int U = 4;
      for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); i0 < cnt; i0 += U * stride) {
        uint64_t bv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint64_t i = i0 + (uint64_t)u * stride + lane;
          bv[u] = i < cnt ? abs_bits((double)coefs<T>(out)[base + i]) : ~0ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const uint64_t i = i0 + (uint64_t)u * stride + lane;
          const uint64_t b = bv[u];
          // the identity is the first string of region (0, 0)
          const bool want = i < cnt && b >= lo && b < hi && !(c == 0 && e == 0 && i == 0);
          const uint64_t mk = __ballot(want);
          if (mk == 0) continue;
          unsigned long long first = 0;
          if (lane == 0) first = atomicAdd((unsigned long long*)&ctl->cand_count, (unsigned long long)__popcll(mk));
          first = __shfl(first, 0, 64);
          if (want) {
            const unsigned long long slot = first + (unsigned long long)__popcll(mk & ((1ull << lane) - 1ull));
            if (slot < sel.cap) {
              sel.cand_bits[slot] = b;
              sel.cand_idx[slot] = base + i;
            } else {
              atomicMax(&ctl->error, kErrCapacity);
            }
          }
        }
      }
    }
}

// Exact K-th value among the candidates (radix select on the |c| bits) and,
// for ties at that value, the largest canonical key still kept.
template <int NW>
__global__ __launch_bounds__(1024) void select_exact(Side out, Filter* filt_out, Ctl* ctl, SelBuf sel,
                                                     RepPos rp) {
  __shared__ uint32_t h[2048];
  __shared__ uint64_t scr[1024];
  __shared__ int s_bin;
  __shared__ uint64_t s_above;
  __shared__ uint32_t s_cnt0;
  __shared__ unsigned long long s_ntie;
  // candidates left after the first radix pass, when few enough (bits, index)
  constexpr uint32_t kLdsCand = 4096;
  __shared__ uint64_t lb[kLdsCand];
  __shared__ uint32_t li[kLdsCand];
  __shared__ uint32_t s_nl;
  if (ctl->error || ctl->halt || ctl->sel_need == 0) return;
  const int tid = threadIdx.x;
  const uint64_t m = ctl->cand_count < sel.cap ? ctl->cand_count : sel.cap;
  bool in_lds = false;
  uint32_t nl = 0;
  uint64_t need = ctl->sel_need;
  // every candidate lies in [sel_lo, sel_hi): the bits above the highest bit
  // in which sel_lo and sel_hi - 1 differ are common, so the radix passes
  // start below them (up to 11 bits per pass)
  const uint64_t diff = ctl->sel_lo ^ (ctl->sel_hi - 1ull);
  int rem = diff ? 64 - __clzll((long long)diff) : 0;
  uint64_t mask = rem >= 64 ? 0ull : ~((1ull << rem) - 1ull);
  uint64_t prefix = ctl->sel_lo & mask;
  uint32_t count_eq = (uint32_t)m;
  while (rem > 0) {
    const int wbits = rem >= 11 ? 11 : rem;
    const int sh = rem - wbits;
    rem = sh;
    const int nb = 1 << wbits;
    const uint64_t dm = (uint64_t)nb - 1ull;
    for (int i = tid; i < 2048; i += blockDim.x) h[i] = 0;
    if (tid == 0) {
      s_bin = -1;
      s_above = 0;
    }
    __syncthreads();
    if (in_lds) {
      for (uint32_t i = tid; i < nl; i += blockDim.x) {
        const uint64_t b = lb[i];
        if ((b & mask) == prefix) atomicAdd(&h[(b >> sh) & dm], 1u);
      }
    } else {
      for (uint64_t i = tid; i < m; i += blockDim.x) {
        const uint64_t b = sel.cand_bits[i];
        if ((b & mask) == prefix) atomicAdd(&h[(b >> sh) & dm], 1u);
      }
    }
    __syncthreads();
    find_from_top(h, nb, 0, need, scr, &s_bin, &s_above);
    const int d = s_bin < 0 ? 0 : s_bin;
    need -= (s_bin < 0 ? 0 : s_above);
    count_eq = h[d];
    prefix |= (uint64_t)d << sh;
    mask |= dm << sh;
    __syncthreads();
    if (!in_lds && count_eq <= kLdsCand) {
      // keep only the candidates of the chosen digit, in LDS
      if (tid == 0) s_nl = 0;
      __syncthreads();
      for (uint64_t i = tid; i < m; i += blockDim.x) {
        const uint64_t b = sel.cand_bits[i];
        if ((b & mask) == prefix) {
          const uint32_t slot = atomicAdd(&s_nl, 1u);
          lb[slot] = b;
          li[slot] = (uint32_t)i;
        }
      }
      __syncthreads();
      nl = s_nl;
      in_lds = true;
    }
  }
  const uint64_t kth = prefix;
  const uint32_t need_eq = (uint32_t)need;
  if (tid == 0) {
    filt_out->kth_bits = kth;
    filt_out->ref_bits = kth;
    filt_out->tie_active = 0;
    s_ntie = 0;
  }
  __syncthreads();
  if (count_eq <= need_eq) return;
  // ties: gather canonical keys of the elements equal to kth
  const uint64_t mt = in_lds ? nl : m;
  for (uint64_t i = tid; i < mt; i += blockDim.x) {
    if ((in_lds ? lb[i] : sel.cand_bits[i]) != kth) continue;
    Key<NW> k = load_key<NW>(out, sel.cand_idx[in_lds ? li[i] : i]);
    Key<NW> ck = to_canonical(k, rp.pos, rp.nbits);
    const unsigned long long slot = atomicAdd(&s_ntie, 1ull);
    for (int q = 0; q < NW; ++q) sel.tie_keys[slot * NW + q] = ck.w[q];
  }
  __syncthreads();
  const uint64_t nt = s_ntie;
  // MSB-first radix selection (8-bit digits, X words before Z words) of
  // the need_eq-th smallest canonical key
  constexpr int W = NW / 2;
  const int n = rp.nbits / 2;
  const int ndig = (n + 7) / 8;  // digits per part; bits above n are zero in every key
  Key<NW> pre, msk;
  for (int q = 0; q < NW; ++q) pre.w[q] = msk.w[q] = 0;
  uint64_t needk = need_eq;
  for (int part = 0; part < 2; ++part) {
    for (int d = ndig - 1; d >= 0; --d) {
      const int word = part * W + (d >> 3);
      const int sh = 8 * (d & 7);
      for (int i = tid; i < 256; i += blockDim.x) h[i] = 0;
      if (tid == 0) {
        s_cnt0 = 0;
        s_bin = -1;
        s_above = 0;
      }
      __syncthreads();
      uint32_t local = 0;
      for (uint64_t i = tid; i < nt; i += blockDim.x) {
        bool match = true;
        for (int q = 0; q < NW; ++q) match = match && ((sel.tie_keys[i * NW + q] & msk.w[q]) == pre.w[q]);
        if (match) {
          atomicAdd(&h[(sel.tie_keys[i * NW + word] >> sh) & 0xffull], 1u);
          ++local;
        }
      }
      if (local) atomicAdd(&s_cnt0, local);
      __syncthreads();
      // the needk-th smallest is the (M - needk + 1)-th largest of the M matches
      const uint64_t M = s_cnt0;
      find_from_top(h, 256, 0, M - needk + 1, scr, &s_bin, &s_above);
      const int bsel = s_bin < 0 ? 0 : s_bin;
      const uint64_t below = M - s_above - h[bsel];
      needk -= below;
      pre.w[word] |= (uint64_t)bsel << sh;
      msk.w[word] |= 0xffull << sh;
      __syncthreads();
    }
  }
  if (tid == 0) {
    filt_out->tie_active = 1;
    for (int q = 0; q < NW; ++q) filt_out->tie_key[q] = pre.w[q];
  }
}

// <O> = sum_j o_j a_{P_j}: binary search of every observable string in its
// class regions, filter and normalise, compensated (TwoSum) reduction in a
// fixed order.

template <int NW, typename T>
__global__ __launch_bounds__(256) void observe_kernel(Side s, const Plan* plan, const Filter* filt,
                                                      RepPos rp, const uint64_t* ox, const uint64_t* oz,
                                                      const double* oc, int32_t m, double* result) {
  __shared__ double ssum[256], scmp[256];
  const int tid = threadIdx.x;
  const Plan& p = *plan;
  const Filter f = *filt;
  constexpr int W = NW / 2;
  const int n = rp.nbits / 2;
  double acc = 0.0, comp = 0.0;
  for (int j = tid; j < m; j += blockDim.x) {
    Key<NW> k;
    for (int q = 0; q < NW; ++q) k.w[q] = 0;
    for (int qb = 0; qb < n; ++qb) {
      if ((ox[(size_t)j * W + (qb >> 6)] >> (qb & 63)) & 1ull) xor_bit(k, rp.pos[qb], 1ull);
      if ((oz[(size_t)j * W + (qb >> 6)] >> (qb & 63)) & 1ull) xor_bit(k, rp.pos[n + qb], 1ull);
    }
    const int e = class_of(k, rp.nbits, p.we);
    double a = 0.0;
    for (int c = 0; c < (1 << p.wc); ++c) {
      uint64_t lo = p.base[c][e], hi = p.base[c][e] + p.cnt[c][e];
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (key_less(load_key<NW>(s, mid), k))
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo < p.base[c][e] + p.cnt[c][e] && key_eq(load_key<NW>(s, lo), k)) {
        const T cs = coefs<T>(s)[lo];
        if (survives(k, (double)cs, f, rp.pos, rp.nbits)) a = (double)normalised<T>(cs, f.cI);
      }
    }
    double term = __dmul_rn(oc[j], a);
    double sres, err;
    two_sum(acc, term, sres, err);
    acc = sres;
    comp = __dadd_rn(comp, err);
  }
  ssum[tid] = acc;
  scmp[tid] = comp;
  __syncthreads();
  for (int w2 = blockDim.x / 2; w2 > 0; w2 >>= 1) {
    if (tid < w2) {
      double sres, err;
      two_sum(ssum[tid], ssum[tid + w2], sres, err);
      ssum[tid] = sres;
      scmp[tid] = __dadd_rn(__dadd_rn(scmp[tid], scmp[tid + w2]), err);
    }
    __syncthreads();
  }
  if (tid == 0) *result = __dadd_rn(ssum[0], scmp[0]);
}

// Copy every surviving string (canonical x/z words, normalised coefficient)
// to the export buffers in arbitrary order.
template <int NW, typename T>
__global__ void export_kernel(Side s, const Plan* plan, const Filter* filt, RepPos rp, uint64_t* ex,
                              uint64_t* ez, double* ec, unsigned long long* count, uint64_t limit) {
  const Plan& p = *plan;
  const Filter f = *filt;
  constexpr int W = NW / 2;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (int c = 0; c < (1 << p.wc); ++c)
    for (int e = 0; e < (1 << p.we); ++e) {
      for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.cnt[c][e]; i += stride) {
        const uint64_t idx = p.base[c][e] + i;
        Key<NW> k = load_key<NW>(s, idx);
        const T cs = coefs<T>(s)[idx];
        if (!survives(k, (double)cs, f, rp.pos, rp.nbits)) continue;
        Key<NW> ck = to_canonical(k, rp.pos, rp.nbits);
        const unsigned long long slot = atomicAdd(count, 1ull);
        if (slot >= limit) continue;
        for (int q = 0; q < W; ++q) {
          ex[slot * W + q] = ck.w[q];
          ez[slot * W + q] = ck.w[W + q];
        }
        ec[slot] = (double)normalised<T>(cs, f.cI);
      }
    }
}

// ---------------------------------------------------------------------------
// Reverse sweep support.

// Copy a stored state into a packed layout: region (c, e) at the running sum
// of the counts of the regions before it (c major, e minor), so the state
// occupies exactly as many elements as it holds.
template <int NW, typename T>
__global__ void pack_kernel(Side src, const Plan* __restrict__ plan_src, Side dst, Plan* __restrict__ plan_dst) {
  const Plan p = *plan_src;
  const int nc = 1 << p.wc, ne = 1 << p.we;
  uint64_t nb[kMaxClasses][kMaxClasses];
  uint64_t acc = 0;
  for (int c = 0; c < kMaxClasses; ++c)
    for (int e = 0; e < kMaxClasses; ++e) {
      nb[c][e] = acc;
      if (c < nc && e < ne) acc += p.cnt[c][e];
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Plan q = p;
    for (int c = 0; c < kMaxClasses; ++c)
      for (int e = 0; e < kMaxClasses; ++e) q.base[c][e] = nb[c][e];
    *plan_dst = q;
  }
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (int c = 0; c < nc; ++c)
    for (int e = 0; e < ne; ++e) {
      const uint64_t sb = p.base[c][e], db = nb[c][e], cnt = p.cnt[c][e];
      for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
#pragma unroll
        for (int q = 0; q < NW; ++q) dst.kw[q][db + i] = src.kw[q][sb + i];
        coefs<T>(dst)[db + i] = coefs<T>(src)[sb + i];
      }
    }
}

// lambda = dL/da for L = sum_j o_j a[P_j]: o_j at the position of every
// observable string the state holds (and keeps), zero elsewhere.
template <int NW>
__global__ __launch_bounds__(256) void seed_kernel(Side s, const Plan* plan, const Filter* filt, RepPos rp,
                                                   const uint64_t* ox, const uint64_t* oz, const double* oc,
                                                   int32_t m, double* lam) {
  const Plan& p = *plan;
  const Filter f = *filt;
  constexpr int W = NW / 2;
  const int n = rp.nbits / 2;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    Key<NW> k;
    for (int q = 0; q < NW; ++q) k.w[q] = 0;
    for (int qb = 0; qb < n; ++qb) {
      if ((ox[(size_t)j * W + (qb >> 6)] >> (qb & 63)) & 1ull) xor_bit(k, rp.pos[qb], 1ull);
      if ((oz[(size_t)j * W + (qb >> 6)] >> (qb & 63)) & 1ull) xor_bit(k, rp.pos[n + qb], 1ull);
    }
    const int e = class_of(k, rp.nbits, p.we);
    for (int c = 0; c < (1 << p.wc); ++c) {
      uint64_t lo = p.base[c][e], hi = p.base[c][e] + p.cnt[c][e];
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (key_less(load_key<NW>(s, mid), k))
          lo = mid + 1;
        else
          hi = mid;
      }
      if (lo < p.base[c][e] + p.cnt[c][e] && key_eq(load_key<NW>(s, lo), k)) {
        if (survives(k, coefs<double>(s)[lo], f, rp.pos, rp.nbits)) atomicAdd(&lam[lo], oc[j]);
      }
    }
  }
}

// dL/dtheta of the gate and sum lambda a of its input, from the per-tile
// partials in tile order (compensated); the ticket is rearmed.
__global__ __launch_bounds__(256) void adj_reduce_kernel(const double* part, const uint64_t* ntiles,
                                                         double* dtheta_out, double* s_out, Ctl* ctl) {
  __shared__ double r[4][256];
  const int tid = threadIdx.x;
  const uint64_t nt = *ntiles;
  const uint64_t per = (nt + 255) / 256;
  double st = 0.0, ct = 0.0, ss = 0.0, cs = 0.0;
  for (uint64_t q = 0; q < per; ++q) {
    const uint64_t t = (uint64_t)tid * per + q;
    if (t >= nt) break;
    double sres, err;
    two_sum(st, part[4 * t], sres, err);
    st = sres;
    ct = __dadd_rn(__dadd_rn(ct, err), part[4 * t + 1]);
    two_sum(ss, part[4 * t + 2], sres, err);
    ss = sres;
    cs = __dadd_rn(__dadd_rn(cs, err), part[4 * t + 3]);
  }
  r[0][tid] = st;
  r[1][tid] = ct;
  r[2][tid] = ss;
  r[3][tid] = cs;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      double sres, err;
      two_sum(r[0][tid], r[0][tid + h], sres, err);
      r[0][tid] = sres;
      r[1][tid] = __dadd_rn(__dadd_rn(r[1][tid], r[1][tid + h]), err);
      two_sum(r[2][tid], r[2][tid + h], sres, err);
      r[2][tid] = sres;
      r[3][tid] = __dadd_rn(__dadd_rn(r[3][tid], r[3][tid + h]), err);
    }
    __syncthreads();
  }
  if (tid == 0) {
    *dtheta_out = __dadd_rn(r[0][0], r[1][0]);
    *s_out = __dadd_rn(r[2][0], r[3][0]);
    ctl->ticket = 0;
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
// Gate kernel shapes (threads per workgroup, merged elements per tile for
// one- and two-word keys).  Shape 0: one 1024-thread workgroup per CU with
// large tiles (large states); shape 1: two 512-thread workgroups per CU with
// half-size tiles (more tiles in flight for small states).  The tile LDS of
// either shape fits the CU's 160 KB at its occupancy.
template <int SHAPE>
struct GateShape;
template <>
struct GateShape<0> {
  static constexpr int block = 1024, wgs_per_cu = 1;
  template <int NW>
  static constexpr int tile() {
    return NW == 2 ? 4000 : 2000;
  }
};
template <>
struct GateShape<1> {
  static constexpr int block = 512, wgs_per_cu = 2;
  template <int NW>
  static constexpr int tile() {
    return NW == 2 ? 2000 : 1500;
  }
};

int gate_tile(int nw, int shape) {
  if (shape == 1) return nw == 2 ? GateShape<1>::tile<2>() : GateShape<1>::tile<4>();
  return nw == 2 ? GateShape<0>::tile<2>() : GateShape<0>::tile<4>();
}
int gate_min_tile(int nw) { return std::min(gate_tile(nw, 0), gate_tile(nw, 1)); }
int gate_wgs_per_cu(int shape) { return shape == 1 ? GateShape<1>::wgs_per_cu : GateShape<0>::wgs_per_cu; }

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

hipError_t launch_init(int nw, int f32, Side s0, Plan* plan, Filter* filt, Ctl* ctl, int w0, hipStream_t st) {
  ITPP_DISPATCH(nw, f32,
                hipLaunchKernelGGL((init_kernel<NWC, TC>), dim3(1), dim3(64), 0, st, s0, plan, filt, ctl, w0));
  return hipGetLastError();
}

hipError_t launch_partition(int nw, const GateParams& gp, Side in, const Plan* plan_in, Ctl* ctl, uint64_t* part,
                            hipStream_t st) {
  // eight tile boundaries per wavefront, four wavefronts per block
  const uint64_t nb = gp.status_cap + kMaxClasses;
  const int pgrid = (int)((nb + 31) / 32);
  if (nw == 2)
    hipLaunchKernelGGL(partition_kernel<2>, dim3(pgrid), dim3(256), 0, st, gp, in, plan_in, part, ctl);
  else
    hipLaunchKernelGGL(partition_kernel<4>, dim3(pgrid), dim3(256), 0, st, gp, in, plan_in, part, ctl);
  return hipGetLastError();
}

template <int SHAPE>
void launch_gate_shape(int nw, int f32, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                       Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part,
                       int grid, hipStream_t st) {
  using S = GateShape<SHAPE>;
  const AdjArgs none{};
  ITPP_DISPATCH(nw, f32,
                hipLaunchKernelGGL((gate_kernel<NWC, S::block, S::template tile<NWC>(), TC, false>), dim3(grid),
                                   dim3(S::block), 0, st, gp, in, out, plan_in, plan_out, filt_in,
                                   (const uint64_t*)part, ctl, status, none));
}

hipError_t launch_gate(int nw, int f32, int shape, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                       Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part,
                       int grid, hipStream_t st) {
  if (shape == 1)
    launch_gate_shape<1>(nw, f32, gp, in, out, plan_in, plan_out, filt_in, ctl, status, part, grid, st);
  else
    launch_gate_shape<0>(nw, f32, gp, in, out, plan_in, plan_out, filt_in, ctl, status, part, grid, st);
  return hipGetLastError();
}

hipError_t launch_adjoint_gate(int nw, const GateParams& gp, Side in, const Plan* plan_in, Plan* plan_scratch,
                               const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part,
                               const AdjArgs& adj, int grid, hipStream_t st) {
  using S = GateShape<0>;
  const Side none{};
  if (nw == 2)
    hipLaunchKernelGGL((gate_kernel<2, S::block, S::tile<2>(), double, true>), dim3(grid), dim3(S::block), 0, st,
                       gp, in, none, plan_in, plan_scratch, filt_in, (const uint64_t*)part, ctl, status, adj);
  else
    hipLaunchKernelGGL((gate_kernel<4, S::block, S::tile<4>(), double, true>), dim3(grid), dim3(S::block), 0, st,
                       gp, in, none, plan_in, plan_scratch, filt_in, (const uint64_t*)part, ctl, status, adj);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const double* part, const uint64_t* ntiles, double* dtheta_out, double* s_out,
                             Ctl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(adj_reduce_kernel, dim3(1), dim3(256), 0, st, part, ntiles, dtheta_out, s_out, ctl);
  return hipGetLastError();
}

hipError_t launch_pack(int nw, int f32, Side src, const Plan* plan_src, Side dst, Plan* plan_dst, int grid,
                       hipStream_t st) {
  ITPP_DISPATCH(nw, f32,
                hipLaunchKernelGGL((pack_kernel<NWC, TC>), dim3(grid), dim3(256), 0, st, src, plan_src, dst,
                                   plan_dst));
  return hipGetLastError();
}

hipError_t launch_seed(int nw, Side s, const Plan* plan, const Filter* filt, const RepPos& rp, const uint64_t* ox,
                       const uint64_t* oz, const double* oc, int32_t m, double* lam, hipStream_t st) {
  const int grid = (m + 255) / 256 > 0 ? (m + 255) / 256 : 1;
  if (nw == 2)
    hipLaunchKernelGGL(seed_kernel<2>, dim3(grid), dim3(256), 0, st, s, plan, filt, rp, ox, oz, oc, m, lam);
  else
    hipLaunchKernelGGL(seed_kernel<4>, dim3(grid), dim3(256), 0, st, s, plan, filt, rp, ox, oz, oc, m, lam);
  return hipGetLastError();
}

hipError_t launch_prepare(Plan* plan_out, Ctl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(prepare_kernel, dim3(1), dim3(1024), 0, st, plan_out, ctl);
  return hipGetLastError();
}

hipError_t launch_select(int nw, int f32, Side out, const Plan* plan_out, const Filter* filt_in,
                         Filter* filt_out, Plan* plan_next, Ctl* ctl, SelBuf sel, const RepPos& rp,
                         int64_t K, int cap_fail, int spec, uint64_t serial, int grid, hipStream_t st) {
  hipLaunchKernelGGL(select_decide, dim3(1), dim3(1024), 0, st, filt_in, filt_out, plan_next, ctl, K,
                     cap_fail, spec, serial);
  ITPP_DISPATCH(nw, f32, {
    hipLaunchKernelGGL((select_coarse_hist<NWC, TC>), dim3(grid / 4 > 0 ? grid / 4 : 1), dim3(256), 0, st, out,
                       plan_out, ctl);
    hipLaunchKernelGGL((select_collect<NWC, TC>), dim3(grid), dim3(256), 0, st, out, plan_out, ctl, sel);
    hipLaunchKernelGGL(select_exact<NWC>, dim3(1), dim3(1024), 0, st, out, filt_out, ctl, sel, rp);
  });
  return hipGetLastError();
}

hipError_t launch_observe(int nw, int f32, Side s, const Plan* plan, const Filter* filt, const RepPos& rp,
                          const uint64_t* ox, const uint64_t* oz, const double* oc, int32_t m,
                          double* result, Ctl* ctl, hipStream_t st) {
  (void)ctl;
  ITPP_DISPATCH(nw, f32,
                hipLaunchKernelGGL((observe_kernel<NWC, TC>), dim3(1), dim3(256), 0, st, s, plan, filt, rp, ox, oz,
                                   oc, m, result));
  return hipGetLastError();
}

hipError_t launch_export(int nw, int f32, Side s, const Plan* plan, const Filter* filt, const RepPos& rp,
                         uint64_t* ex, uint64_t* ez, double* ec, unsigned long long* count, uint64_t limit,
                         int grid, hipStream_t st) {
  ITPP_DISPATCH(nw, f32,
                hipLaunchKernelGGL((export_kernel<NWC, TC>), dim3(grid), dim3(256), 0, st, s, plan, filt, rp, ex,
                                   ez, ec, count, limit));
  return hipGetLastError();
}

}  // namespace itpp
