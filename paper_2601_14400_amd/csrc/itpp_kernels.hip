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

template <int NW>
__device__ __forceinline__ int get_bit(const Key<NW>& k, int p) {
  return (int)((k.w[p >> 6] >> (p & 63)) & 1ull);
}

template <int NW>
__device__ __forceinline__ void flip_bit(Key<NW>& k, int p) {
  k.w[p >> 6] ^= (1ull << (p & 63));
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
  const int b = get_bit(k, p);
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
  if (b) r.w[(nbits - 1) >> 6] |= 1ull << ((nbits - 1) & 63);
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
      c.w[word] |= 1ull << bit;
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

__device__ inline ClassView make_view(const Plan& p, int cls) {
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
  if (nc < kMaxClasses) v.start[nc] = acc;
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

// End (exclusive) of output region (c, e): the next region's base in the
// (c major, e minor) layout, or the total for the last region.
__device__ __forceinline__ uint64_t region_end(const uint64_t (*ob)[kMaxClasses], int c, int e, int ncls,
                                               int ncls1) {
  (void)ncls;
  (void)ncls1;
  int cc = c, ee = e + 1;
  if (ee == kMaxClasses) {
    ee = 0;
    ++cc;
  }
  if (cc == kMaxClasses) return ob[kMaxClasses][0];
  return ob[cc][ee];
}

// ---------------------------------------------------------------------------
// The gate kernel.
template <int NW, int BLOCK, int TILE>
struct GateSmem {
  static constexpr int CAPT = TILE + 2;
  uint64_t key[NW][CAPT];
  double coef[CAPT];
  uint8_t flag[CAPT];      // bit0 survive, bit1 commuting
  uint64_t vs[CAPT + 1];   // self one-hot (16-bit lanes per next class), then exclusive scan
  uint64_t vb[CAPT + 1];   // branch one-hot, then exclusive scan
  uint64_t wa[BLOCK / 64], wb[BLOCK / 64];
  uint32_t hist[kHistBins];
  uint32_t ncnt[kMaxClasses * kMaxClasses];
  uint64_t out_base[kMaxClasses + 1][kMaxClasses];  // row kMaxClasses holds the total
  uint32_t excl[2 * kMaxClasses];
  uint64_t i0, j0, i1, j1;
  uint32_t tile;
  uint32_t nwritten;
  ClassView views[kMaxClasses];
  uint64_t tiles_before[kMaxClasses / 2 + 1];
};

template <int NW>
__device__ inline uint64_t corank(const Side& in, const ClassView& A, const ClassView& B, uint64_t d,
                                  int nbits, int w) {
  const uint64_t nA = A.size(), nB = B.size();
  uint64_t lo = d > nB ? d - nB : 0;
  uint64_t hi = d < nA ? d : nA;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    Key<NW> a = load_key<NW>(in, A.phys(mid));
    Key<NW> b = xor_top(load_key<NW>(in, B.phys(d - mid - 1)), nbits, w);
    if (!key_less(b, a))  // a <= b'
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <int NW, int BLOCK, int TILE>
__global__ __launch_bounds__(BLOCK) void gate_kernel(GateParams gp, Side in, Side out,
                                                      const Plan* __restrict__ plan_in,
                                                      Plan* __restrict__ plan_out,
                                                      const Filter* __restrict__ filt_in,
                                                      Ctl* __restrict__ ctl,
                                                      TileStatus* __restrict__ status) {
  using Smem = GateSmem<NW, BLOCK, TILE>;
  __shared__ Smem sm;
  constexpr int ITEMS = (TILE + 2 + BLOCK - 1) / BLOCK;
  const int tid = threadIdx.x;
  const Plan pin = *plan_in;
  const Filter fin = *filt_in;
  const int nbits = gp.nbits;
  const int w = gp.w;
  const int ncls = 1 << w;
  const int full = ncls - 1;
  const int ncls1 = 1 << gp.w1;
  const int njoin = ncls >> 1;

  for (int i = tid; i < kHistBins; i += BLOCK) sm.hist[i] = 0;
  if (tid < kMaxClasses * kMaxClasses) sm.ncnt[tid] = 0;
  if (tid == 0) {
    // output region capacities: cap(c,e) = n[c][e] + n[~c][e ^ ov]
    uint64_t acc = 0;
    for (int c = 0; c < kMaxClasses; ++c)
      for (int e = 0; e < kMaxClasses; ++e) {
        sm.out_base[c][e] = acc;
        if (c < ncls && e < ncls1) acc += (uint64_t)pin.ncnt[c][e] + (uint64_t)pin.ncnt[c ^ full][e ^ gp.ov];
      }
    for (int e = 0; e < kMaxClasses; ++e) sm.out_base[kMaxClasses][e] = acc;
    if (acc > gp.cap_elems) atomicMax(&ctl->error, kErrCapacity);
    if (blockIdx.x == 0) {
      for (int c = 0; c < kMaxClasses; ++c)
        for (int e = 0; e < kMaxClasses; ++e) plan_out->base[c][e] = sm.out_base[c][e];
      plan_out->wc = w;
      plan_out->we = gp.w1;
    }
    sm.nwritten = 0;
  }
  if (tid == 0) {
    for (int c = 0; c < kMaxClasses; ++c) sm.views[c] = make_view(pin, c < ncls ? c : 0);
    sm.tiles_before[0] = 0;
    for (int j = 0; j < kMaxClasses / 2; ++j) {
      uint64_t L = 0;
      if (j < njoin) L = sm.views[j].size() + sm.views[j ^ full].size();
      sm.tiles_before[j + 1] = sm.tiles_before[j] + (L + TILE - 1) / TILE;
    }
  }
  __syncthreads();
  const uint64_t total_tiles = sm.tiles_before[njoin];
  if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kErrNone) return;

  uint64_t my_written = 0;
  for (;;) {
    if (tid == 0) sm.tile = atomicAdd(&ctl->ticket, 1u);
    __syncthreads();
    const uint64_t t = sm.tile;
    if (t >= total_tiles) break;
    if (t >= gp.status_cap) {
      if (tid == 0) atomicMax(&ctl->error, kErrCapacity);
      break;
    }
    int j = 0;
    while (j + 1 < njoin && t >= sm.tiles_before[j + 1]) ++j;
    const uint64_t tl = t - sm.tiles_before[j];
    const int cA = j, cB = j ^ full;
    const ClassView& VA = sm.views[cA];
    const ClassView& VB = sm.views[cB];
    const uint64_t nA = VA.size(), nB = VB.size();
    const uint64_t L = nA + nB;
    const uint64_t d0 = tl * TILE;
    const uint64_t d1 = (d0 + TILE < L) ? d0 + TILE : L;
    // merge-path co-ranks, pairs kept in the earlier tile
    if (tid == 0 || tid == 64) {
      const uint64_t d = (tid == 0) ? d0 : d1;
      uint64_t i = corank<NW>(in, VA, VB, d, nbits, w);
      uint64_t jj = d - i;
      if (i > 0 && jj < nB) {
        Key<NW> a = load_key<NW>(in, VA.phys(i - 1));
        Key<NW> b = xor_top(load_key<NW>(in, VB.phys(jj)), nbits, w);
        if (key_eq(a, b)) jj += 1;
      }
      if (tid == 0) {
        sm.i0 = i;
        sm.j0 = jj;
      } else {
        sm.i1 = i;
        sm.j1 = jj;
      }
    }
    __syncthreads();
    const uint64_t i0 = sm.i0, j0 = sm.j0;
    const int nAt = (int)(sm.i1 - sm.i0);
    const int nBt = (int)(sm.j1 - sm.j0);
    const int nt = nAt + nBt;

    // load, filter, normalise
    for (int x = tid; x < nt; x += BLOCK) {
      const bool isA = x < nAt;
      const uint64_t p = isA ? VA.phys(i0 + x) : VB.phys(j0 + (x - nAt));
      Key<NW> k = load_key<NW>(in, p);
      const double cs = in.coef[p];
      const bool sv = survives(k, cs, fin, gp.pos_in, nbits);
      const bool comm = !anticommutes(k, gp);
      if (!isA) k = xor_top(k, nbits, w);  // B' = B xor Q lives in class cA's key space
#pragma unroll
      for (int q = 0; q < NW; ++q) sm.key[q][x] = k.w[q];
      sm.coef[x] = cs / fin.cI;
      sm.flag[x] = (uint8_t)((sv ? 1 : 0) | (comm ? 2 : 0));
    }
    __syncthreads();

    // partner search, outputs, one-hot class vectors
    double vself[ITEMS], vbr[ITEMS];
    uint32_t lbo[ITEMS];
    uint8_t eo[ITEMS];  // low nibble: self class, high nibble: branch class
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int x = tid + it * BLOCK;
      vself[it] = 0.0;
      vbr[it] = 0.0;
      lbo[it] = 0;
      eo[it] = 0;
      uint64_t onehot_s = 0, onehot_b = 0;
      if (x < nt) {
        const bool isA = x < nAt;
        Key<NW> k;
#pragma unroll
        for (int q = 0; q < NW; ++q) k.w[q] = sm.key[q][x];
        // lower bound of k in the other range
        int lo = isA ? nAt : 0;
        int hi = isA ? nt : nAt;
        const int base = lo;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          Key<NW> m;
#pragma unroll
          for (int q = 0; q < NW; ++q) m.w[q] = sm.key[q][mid];
          if (key_less(m, k))
            lo = mid + 1;
          else
            hi = mid;
        }
        const int lb = lo - base;
        lbo[it] = (uint32_t)lb;
        const uint8_t fl = sm.flag[x];
        if (fl & 1) {
          bool paired = false;
          double cp = 0.0;
          if (lo < (isA ? nt : nAt)) {
            Key<NW> m;
#pragma unroll
            for (int q = 0; q < NW; ++q) m.w[q] = sm.key[q][lo];
            if (key_eq(m, k) && (sm.flag[lo] & 1)) {
              paired = true;
              cp = sm.coef[lo];
            }
          }
          const double c = sm.coef[x];
          // own key in this gate's rep
          const Key<NW> own = isA ? k : xor_top(k, nbits, w);
          const Key<NW> brk = isA ? xor_top(k, nbits, w) : k;
          bool hs = false, hb = false;
          if (!(fl & 2)) {
            vself[it] = c;
            hs = fabs(c) > gp.delta;
          } else {
            const int e4 = phase_negative(own, gp);
            if (e4 & 1) atomicMax(&ctl->error, kErrPhase);
            const bool neg = (e4 == 2);  // Q P = -R
            const double t1 = __dmul_rn(gp.ch, c);
            if (paired) {
              double t2 = __dmul_rn(gp.sh, cp);
              if (!neg) t2 = -t2;
              vself[it] = __dadd_rn(t1, t2);
            } else {
              vself[it] = t1;
              double t2 = __dmul_rn(gp.sh, c);
              if (!neg) t2 = -t2;
              vbr[it] = t2;
              hb = fabs(t2) > gp.delta;
            }
            hs = fabs(vself[it]) > gp.delta;
          }
          Key<NW> ks = own, kb = brk;
          for (int m = 0; m < gp.w1; ++m) {
            ks = move_top(ks, gp.mv[m], nbits);
            kb = move_top(kb, gp.mv[m], nbits);
          }
          const int es = class_of(ks, nbits, gp.w1);
          const int eb = class_of(kb, nbits, gp.w1);
          eo[it] = (uint8_t)(es | (eb << 4));
          if (hs) onehot_s = 1ull << (16 * es);
          if (hb) onehot_b = 1ull << (16 * eb);
          if (!hs) vself[it] = 0.0, eo[it] |= 0x08;  // mark no self
          if (!hb) eo[it] |= 0x80;                   // mark no branch
        } else {
          eo[it] = 0x88;
        }
      }
      if (x < TILE + 2) {
        sm.vs[x] = onehot_s;
        sm.vb[x] = onehot_b;
      }
    }
    __syncthreads();
    // exclusive scans over [0, nt) in blocked layout; entry nt = total
    {
      constexpr int PER = ITEMS;
      const int s0 = tid * PER;
      uint64_t la[PER], lb2[PER];
      uint64_t suma = 0, sumb = 0;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int x = s0 + q;
        la[q] = (x < nt) ? sm.vs[x] : 0;
        lb2[q] = (x < nt) ? sm.vb[x] : 0;
        suma += la[q];
        sumb += lb2[q];
      }
      uint64_t pa = suma, pb = sumb, ta, tb;
      block_scan2<BLOCK>(pa, pb, sm.wa, sm.wb, ta, tb);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int x = s0 + q;
        if (x < nt) {
          sm.vs[x] = pa;
          sm.vb[x] = pb;
        }
        pa += la[q];
        pb += lb2[q];
      }
      if (tid == 0) {
        sm.vs[nt] = ta;
        sm.vb[nt] = tb;
      }
    }
    __syncthreads();
    // tile totals per (side, next class) and look-back
    if (tid == 0) {
      const uint64_t As = sm.vs[nAt], Ab = sm.vb[nAt];
      const uint64_t Bs = sm.vs[nt] - As, Bb = sm.vb[nt] - Ab;
      uint32_t agg[2 * kMaxClasses];
      for (int e = 0; e < kMaxClasses; ++e) {
        agg[e] = lane16(As, e) + lane16(Bb, e);                // class cA stream
        agg[kMaxClasses + e] = lane16(Bs, e) + lane16(Ab, e);  // class cB stream
      }
      TileStatus* st = status + t;
      const uint32_t ep = gp.epoch << 2;
      uint32_t excl[2 * kMaxClasses];
      for (int q = 0; q < 2 * kMaxClasses; ++q) excl[q] = 0;
      if (tl == 0) {
        for (int q = 0; q < 2 * kMaxClasses; ++q)
          __hip_atomic_store(&st->incl[q], agg[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&st->flag, ep | 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        for (int q = 0; q < 2 * kMaxClasses; ++q)
          __hip_atomic_store(&st->agg[q], agg[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&st->flag, ep | 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int64_t k = (int64_t)t - 1;
        const int64_t first = (int64_t)sm.tiles_before[j];
        while (k >= first) {
          TileStatus* ps = status + k;
          uint32_t f = 0;
          uint32_t spins = 0;
          for (;;) {
            f = __hip_atomic_load(&ps->flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if ((f >> 2) == gp.epoch && (f & 3u) != 0) break;
            if (++spins > (1u << 26)) {
              atomicMax(&ctl->error, kErrSpin);
              f = ep | 2u;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          if ((f & 3u) == 2u) {
            for (int q = 0; q < 2 * kMaxClasses; ++q)
              excl[q] += __hip_atomic_load(&ps->incl[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          for (int q = 0; q < 2 * kMaxClasses; ++q)
            excl[q] += __hip_atomic_load(&ps->agg[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          --k;
        }
        for (int q = 0; q < 2 * kMaxClasses; ++q)
          __hip_atomic_store(&st->incl[q], excl[q] + agg[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&st->flag, ep | 2u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
      for (int q = 0; q < 2 * kMaxClasses; ++q) sm.excl[q] = excl[q];
      // the last tile of the join publishes the region fill counts
      if (t + 1 == sm.tiles_before[j + 1]) {
        for (int e = 0; e < ncls1; ++e) {
          plan_out->cnt[cA][e] = excl[e] + agg[e];
          plan_out->cnt[cB][e] = excl[kMaxClasses + e] + agg[kMaxClasses + e];
        }
      }
    }
    __syncthreads();
    // write outputs
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
      const int x = tid + it * BLOCK;
      if (x >= nt) continue;
      const uint8_t e = eo[it];
      const bool hs = !(e & 0x08);
      const bool hb = !(e & 0x80);
      if (!hs && !hb) continue;
      const bool isA = x < nAt;
      const int lb = (int)lbo[it];
      Key<NW> k;
#pragma unroll
      for (int q = 0; q < NW; ++q) k.w[q] = sm.key[q][x];
      const Key<NW> own = isA ? k : xor_top(k, nbits, w);
      const Key<NW> brk = isA ? xor_top(k, nbits, w) : k;
      // prefix values at this element and at the partner rank in the other range
      const uint64_t my_s = sm.vs[x], my_b = sm.vb[x];
      uint64_t oth_s, oth_b;
      if (isA) {
        oth_s = sm.vs[nAt + lb] - sm.vs[nAt];
        oth_b = sm.vb[nAt + lb] - sm.vb[nAt];
      } else {
        oth_s = sm.vs[lb];
        oth_b = sm.vb[lb];
      }
      const uint64_t mys = isA ? my_s : my_s - sm.vs[nAt];
      const uint64_t myb = isA ? my_b : my_b - sm.vb[nAt];
      if (hs) {
        const int es = e & 0x7;
        // self output: stream of own class
        const int side = isA ? 0 : 1;
        const int cls = isA ? cA : cB;
        const uint64_t pos = sm.out_base[cls][es] + sm.excl[side * kMaxClasses + es] + lane16(mys, es) +
                             lane16(oth_b, es);
        Key<NW> ks = own;
        for (int m = 0; m < gp.w1; ++m) ks = move_top(ks, gp.mv[m], nbits);
        if (pos >= region_end(sm.out_base, cls, es, ncls, ncls1)) {
          atomicMax(&ctl->error, kErrCapacity);
          continue;
        }
        store_key<NW>(out, pos, ks);
        out.coef[pos] = vself[it];
        if (key_zero(ks)) {
          ctl->cI_out = vself[it];
          ctl->have_cI = 1u;
        } else {
          atomicAdd(&sm.hist[hist_bin(abs_bits(vself[it]))], 1u);
          ++my_written;
        }
        int f = 0;
        for (int b = 0; b < gp.w2; ++b) f |= get_bit(ks, gp.fpos[b]) << b;
        atomicAdd(&sm.ncnt[es * kMaxClasses + f], 1u);
      }
      if (hb) {
        const int eb = (e >> 4) & 0x7;
        const int side = isA ? 1 : 0;
        const int cls = isA ? cB : cA;
        const uint64_t pos = sm.out_base[cls][eb] + sm.excl[side * kMaxClasses + eb] + lane16(myb, eb) +
                             lane16(oth_s, eb);
        Key<NW> kb = brk;
        for (int m = 0; m < gp.w1; ++m) kb = move_top(kb, gp.mv[m], nbits);
        if (pos >= region_end(sm.out_base, cls, eb, ncls, ncls1)) {
          atomicMax(&ctl->error, kErrCapacity);
          continue;
        }
        store_key<NW>(out, pos, kb);
        out.coef[pos] = vbr[it];
        atomicAdd(&sm.hist[hist_bin(abs_bits(vbr[it]))], 1u);
        ++my_written;
        int f = 0;
        for (int b = 0; b < gp.w2; ++b) f |= get_bit(kb, gp.fpos[b]) << b;
        atomicAdd(&sm.ncnt[eb * kMaxClasses + f], 1u);
      }
    }
    __syncthreads();
  }
  // flush per-workgroup statistics
  __syncthreads();
  for (int i = tid; i < kHistBins; i += BLOCK) {
    const uint32_t v = sm.hist[i];
    if (v) atomicAdd(&ctl->hist[i], v);
  }
  if (tid < kMaxClasses * kMaxClasses) {
    const uint32_t v = sm.ncnt[tid];
    if (v) atomicAdd(&plan_out->ncnt[tid / kMaxClasses][tid % kMaxClasses], v);
  }
  if (my_written) atomicAdd(&sm.nwritten, (uint32_t)my_written);
  __syncthreads();
  if (tid == 0 && sm.nwritten)
    atomicAdd((unsigned long long*)&ctl->n_written_nonid, (unsigned long long)sm.nwritten);
}


// ---------------------------------------------------------------------------
// rho = I: one identity string with coefficient 1 (Algorithm 1 initial state).
template <int NW>
__global__ void init_kernel(Side s0, Plan* plan, Filter* filt, Ctl* ctl, int w0) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < NW; ++q) s0.kw[q][0] = 0ull;
  s0.coef[0] = 1.0;
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

// After a gate: check the identity coefficient, decide whether the cap
// binds and locate the histogram bin that holds the K-th value; prepare the
// control block for the next gate.
__global__ void select_decide(const Filter* filt_in, Filter* filt_out, Plan* plan_next, Ctl* ctl,
                              int64_t K, int cap_fail) {
  __shared__ uint32_t h[kHistBins];
  __shared__ uint32_t res_bin, res_need;
  const int tid = threadIdx.x;
  if (ctl->error) return;
  for (int i = tid; i < kHistBins; i += blockDim.x) h[i] = ctl->hist[i];
  __syncthreads();
  const uint64_t nw = ctl->n_written_nonid + 1;  // identity included
  const bool capped = (int64_t)nw > K;
  if (tid == 0) {
    res_bin = 0;
    res_need = 0;
    if (capped) {
      const uint64_t need = (uint64_t)(K - 1);
      uint64_t cum = 0;
      int b = kHistBins - 1;
      for (; b >= 0; --b) {
        if (cum + h[b] >= need) break;
        cum += h[b];
      }
      if (b < 0) b = 0;
      res_bin = (uint32_t)b;
      res_need = (uint32_t)(need - cum);
    }
  }
  __syncthreads();
  for (int i = tid; i < kHistBins; i += blockDim.x) ctl->hist[i] = 0;
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
    f.kth_bits = 0;
    f.tie_active = 0;
    f.n_survivors = capped ? (uint64_t)K : nw;
    *filt_out = f;
    ctl->term_updates += (double)filt_in->n_survivors;
    ctl->gates += 1;
    if (capped) ctl->cap_hit = 1;
    ctl->sel_bin = res_bin;
    ctl->sel_need = capped ? res_need : 0u;
    ctl->cand_count = 0;
    ctl->ticket = 0;
    ctl->n_written_nonid = 0;
    ctl->have_cI = 0;
  }
}

// Collect the stored non-identity elements of the K-th value's bin.
template <int NW>
__global__ void select_collect(Side out, const Plan* plan, Ctl* ctl, SelBuf sel) {
  if (ctl->error || ctl->sel_need == 0) return;
  const uint32_t bin = ctl->sel_bin;
  const Plan p = *plan;
  const int nc = 1 << p.wc, ne = 1 << p.we;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (int c = 0; c < nc; ++c)
    for (int e = 0; e < ne; ++e) {
      const uint64_t base = p.base[c][e];
      const uint64_t cnt = p.cnt[c][e];
      for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cnt; i += stride) {
        const uint64_t idx = base + i;
        const uint64_t b = abs_bits(out.coef[idx]);
        if ((uint32_t)hist_bin(b) != bin) continue;
        Key<NW> k = load_key<NW>(out, idx);
        if (key_zero(k)) continue;
        const unsigned long long slot = atomicAdd((unsigned long long*)&ctl->cand_count, 1ull);
        if (slot < sel.cap) {
          sel.cand_bits[slot] = b;
          sel.cand_idx[slot] = idx;
        } else {
          atomicMax(&ctl->error, kErrCapacity);
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
  __shared__ uint64_t s_prefix, s_mask;
  __shared__ uint32_t s_need, s_digit, s_eq;
  __shared__ uint32_t s_cnt0;
  __shared__ unsigned long long s_ntie;
  if (ctl->error || ctl->sel_need == 0) return;
  const int tid = threadIdx.x;
  const uint64_t m = ctl->cand_count < sel.cap ? ctl->cand_count : sel.cap;
  if (tid == 0) {
    s_prefix = 0;
    s_mask = 0;
    s_need = ctl->sel_need;
  }
  __syncthreads();
  const int shifts[6] = {53, 42, 31, 20, 9, 0};
  const int widths[6] = {11, 11, 11, 11, 11, 9};
  for (int pass = 0; pass < 6; ++pass) {
    const int sh = shifts[pass];
    const uint64_t dm = (1ull << widths[pass]) - 1ull;
    for (int i = tid; i < 2048; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t pre = s_prefix, msk = s_mask;
    for (uint64_t i = tid; i < m; i += blockDim.x) {
      const uint64_t b = sel.cand_bits[i];
      if ((b & msk) == pre) atomicAdd(&h[(b >> sh) & dm], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t need = s_need;
      uint32_t cum = 0;
      int d = (int)dm;
      for (; d >= 0; --d) {
        if (cum + h[d] >= need) break;
        cum += h[d];
      }
      if (d < 0) d = 0;
      s_need = need - cum;
      s_digit = (uint32_t)d;
      s_eq = h[d];
      s_prefix = pre | ((uint64_t)d << sh);
      s_mask = msk | (dm << sh);
    }
    __syncthreads();
  }
  const uint64_t kth = s_prefix;
  const uint32_t need_eq = s_need;
  const uint32_t count_eq = s_eq;
  if (tid == 0) {
    filt_out->kth_bits = kth;
    filt_out->tie_active = 0;
    s_ntie = 0;
  }
  __syncthreads();
  if (count_eq <= need_eq) return;
  // ties: gather canonical keys of the elements equal to kth
  for (uint64_t i = tid; i < m; i += blockDim.x) {
    if (sel.cand_bits[i] != kth) continue;
    Key<NW> k = load_key<NW>(out, sel.cand_idx[i]);
    Key<NW> ck = to_canonical(k, rp.pos, rp.nbits);
    const unsigned long long slot = atomicAdd(&s_ntie, 1ull);
    for (int q = 0; q < NW; ++q) sel.tie_keys[slot * NW + q] = ck.w[q];
  }
  __syncthreads();
  const uint64_t nt = s_ntie;
  // MSB-first selection of the need_eq-th smallest canonical key
  constexpr int W = NW / 2;
  const int n = rp.nbits / 2;
  Key<NW> pre, msk;
  for (int q = 0; q < NW; ++q) pre.w[q] = msk.w[q] = 0;
  uint32_t need = need_eq;
  for (int part = 0; part < 2; ++part) {
    for (int qb = n - 1; qb >= 0; --qb) {
      const int word = part * W + (qb >> 6);
      const uint64_t bit = 1ull << (qb & 63);
      if (tid == 0) s_cnt0 = 0;
      __syncthreads();
      uint32_t local = 0;
      for (uint64_t i = tid; i < nt; i += blockDim.x) {
        bool match = true;
        for (int q = 0; q < NW; ++q) match = match && ((sel.tie_keys[i * NW + q] & msk.w[q]) == pre.w[q]);
        if (match && !(sel.tie_keys[i * NW + word] & bit)) ++local;
      }
      if (local) atomicAdd(&s_cnt0, local);
      __syncthreads();
      const uint32_t c0 = s_cnt0;
      if (c0 < need) {
        need -= c0;
        pre.w[word] |= bit;
      }
      msk.w[word] |= bit;
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
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = __dadd_rn(a, b);
  const double bb = __dsub_rn(s, a);
  e = __dadd_rn(__dsub_rn(a, __dsub_rn(s, bb)), __dsub_rn(b, bb));
}

template <int NW>
__global__ __launch_bounds__(256) void observe_kernel(Side s, const Plan* plan, const Filter* filt,
                                                      RepPos rp, const uint64_t* ox, const uint64_t* oz,
                                                      const double* oc, int32_t m, double* result) {
  __shared__ double ssum[256], scmp[256];
  const int tid = threadIdx.x;
  const Plan p = *plan;
  const Filter f = *filt;
  constexpr int W = NW / 2;
  const int n = rp.nbits / 2;
  double acc = 0.0, comp = 0.0;
  for (int j = tid; j < m; j += blockDim.x) {
    Key<NW> k;
    for (int q = 0; q < NW; ++q) k.w[q] = 0;
    for (int qb = 0; qb < n; ++qb) {
      if ((ox[(size_t)j * W + (qb >> 6)] >> (qb & 63)) & 1ull) {
        const int pp = rp.pos[qb];
        k.w[pp >> 6] |= 1ull << (pp & 63);
      }
      if ((oz[(size_t)j * W + (qb >> 6)] >> (qb & 63)) & 1ull) {
        const int pp = rp.pos[n + qb];
        k.w[pp >> 6] |= 1ull << (pp & 63);
      }
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
        const double cs = s.coef[lo];
        if (survives(k, cs, f, rp.pos, rp.nbits)) a = cs / f.cI;
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
template <int NW>
__global__ void export_kernel(Side s, const Plan* plan, const Filter* filt, RepPos rp, uint64_t* ex,
                              uint64_t* ez, double* ec, unsigned long long* count, uint64_t limit) {
  const Plan p = *plan;
  const Filter f = *filt;
  constexpr int W = NW / 2;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (int c = 0; c < (1 << p.wc); ++c)
    for (int e = 0; e < (1 << p.we); ++e) {
      for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < p.cnt[c][e]; i += stride) {
        const uint64_t idx = p.base[c][e] + i;
        Key<NW> k = load_key<NW>(s, idx);
        const double cs = s.coef[idx];
        if (!survives(k, cs, f, rp.pos, rp.nbits)) continue;
        Key<NW> ck = to_canonical(k, rp.pos, rp.nbits);
        const unsigned long long slot = atomicAdd(count, 1ull);
        if (slot >= limit) continue;
        for (int q = 0; q < W; ++q) {
          ex[slot * W + q] = ck.w[q];
          ez[slot * W + q] = ck.w[W + q];
        }
        ec[slot] = cs / f.cI;
      }
    }
}

// ---------------------------------------------------------------------------
// Host launchers.
constexpr int kBlock = 256;
template <int NW>
struct TileFor;
template <>
struct TileFor<2> {
  static constexpr int value = 1024;
};
template <>
struct TileFor<4> {
  static constexpr int value = 1024;
};

int gate_tile(int nw) { return nw == 2 ? TileFor<2>::value : TileFor<4>::value; }

hipError_t launch_init(int nw, Side s0, Plan* plan, Filter* filt, Ctl* ctl, int w0, hipStream_t st) {
  if (nw == 2)
    hipLaunchKernelGGL(init_kernel<2>, dim3(1), dim3(64), 0, st, s0, plan, filt, ctl, w0);
  else
    hipLaunchKernelGGL(init_kernel<4>, dim3(1), dim3(64), 0, st, s0, plan, filt, ctl, w0);
  return hipGetLastError();
}

hipError_t launch_gate(int nw, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                       Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, int grid,
                       hipStream_t st) {
  if (nw == 2)
    hipLaunchKernelGGL((gate_kernel<2, kBlock, TileFor<2>::value>), dim3(grid), dim3(kBlock), 0, st, gp,
                       in, out, plan_in, plan_out, filt_in, ctl, status);
  else
    hipLaunchKernelGGL((gate_kernel<4, kBlock, TileFor<4>::value>), dim3(grid), dim3(kBlock), 0, st, gp,
                       in, out, plan_in, plan_out, filt_in, ctl, status);
  return hipGetLastError();
}

hipError_t launch_select(int nw, Side out, const Plan* plan_out, const Filter* filt_in,
                         Filter* filt_out, Plan* plan_next, Ctl* ctl, SelBuf sel, const RepPos& rp,
                         int64_t K, int cap_fail, int grid, hipStream_t st) {
  hipLaunchKernelGGL(select_decide, dim3(1), dim3(1024), 0, st, filt_in, filt_out, plan_next, ctl, K,
                     cap_fail);
  if (nw == 2) {
    hipLaunchKernelGGL(select_collect<2>, dim3(grid), dim3(256), 0, st, out, plan_out, ctl, sel);
    hipLaunchKernelGGL(select_exact<2>, dim3(1), dim3(1024), 0, st, out, filt_out, ctl, sel, rp);
  } else {
    hipLaunchKernelGGL(select_collect<4>, dim3(grid), dim3(256), 0, st, out, plan_out, ctl, sel);
    hipLaunchKernelGGL(select_exact<4>, dim3(1), dim3(1024), 0, st, out, filt_out, ctl, sel, rp);
  }
  return hipGetLastError();
}

hipError_t launch_observe(int nw, Side s, const Plan* plan, const Filter* filt, const RepPos& rp,
                          const uint64_t* ox, const uint64_t* oz, const double* oc, int32_t m,
                          double* result, Ctl* ctl, hipStream_t st) {
  (void)ctl;
  if (nw == 2)
    hipLaunchKernelGGL(observe_kernel<2>, dim3(1), dim3(256), 0, st, s, plan, filt, rp, ox, oz, oc, m,
                       result);
  else
    hipLaunchKernelGGL(observe_kernel<4>, dim3(1), dim3(256), 0, st, s, plan, filt, rp, ox, oz, oc, m,
                       result);
  return hipGetLastError();
}

hipError_t launch_export(int nw, Side s, const Plan* plan, const Filter* filt, const RepPos& rp,
                         uint64_t* ex, uint64_t* ez, double* ec, unsigned long long* count, uint64_t limit,
                         int grid, hipStream_t st) {
  if (nw == 2)
    hipLaunchKernelGGL(export_kernel<2>, dim3(grid), dim3(256), 0, st, s, plan, filt, rp, ex, ez, ec, count,
                       limit);
  else
    hipLaunchKernelGGL(export_kernel<4>, dim3(grid), dim3(256), 0, st, s, plan, filt, rp, ex, ez, ec, count,
                       limit);
  return hipGetLastError();
}

}  // namespace itpp
