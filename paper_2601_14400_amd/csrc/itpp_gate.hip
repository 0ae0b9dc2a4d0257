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
#include <type_traits>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "itpp_device.h"

namespace itpp {

// ---------------------------------------------------------------------------
// Merge-path partition: eight tile boundaries per wavefront, each searched
// by a group of 8 lanes (8-ary search of the co-rank: the number of class-A
// strings among the first d of the merged sequence, A first on equal keys;
// few probes per level keep the scattered key reads small), then a pair
// split by the boundary is moved into the earlier tile.
template <int NW>
__global__ __launch_bounds__(256) void partition_kernel(GateParams gp, Side in, const Plan* __restrict__ plan_in,
                                                         uint64_t* __restrict__ part, Ctl* __restrict__ ctl,
                                                         TileStatus* __restrict__ status) {
  __shared__ JoinLayout L;
  __shared__ Plan s_pin;
  plan_to_lds(&s_pin, plan_in, threadIdx.x);
  __syncthreads();
  if (threadIdx.x == 0) make_layout(L, &s_pin, gp.w, gp.tile);
  __syncthreads();
  if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kErrNone || ctl->halt) return;
  // the look-back records carry 12-bit epoch tags that repeat every 4095
  // gates: clear them all every kStatusClearEvery gates (before the gate
  // kernel of this gate reads them; nothing else runs in between)
  if (ctl->epoch % kStatusClearEvery == 0) {
    const uint64_t nwords = (uint64_t)kStatusWords * gp.status_cap;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) status[i] = 0ull;
  }
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
      Key<NW> bb = xor_mask(load_key<NW>(in, VB.phys(d - i - 1)), gp.topm);
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
      Key<NW> bb = xor_mask(load_key<NW>(in, VB.phys(jj)), gp.topm);
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
//
// RT = true applies the real-time rule of Sec. II.B instead (gp.ch = cos,
// gp.sh = sin): anticommuting strings branch, cos(theta) P + i sin(theta) Q P,
// with Q P = i^k R for odd k; commuting ones pass unchanged.  Info bit 1 then
// marks the branching (anticommuting) strings and the merge-join is the same.
template <int NW, int BLOCK, int TILE, typename T, bool ADJ, bool RT = false>
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
  const uint32_t epoch = ctl->epoch;
  const T ch = (T)gp.ch, sh = (T)gp.sh;
  const int nbits = gp.nbits;
  const int w = gp.w;
  const int ncls = 1 << w;
  const int full = ncls - 1;
  const int ncls1 = 1 << gp.w1;
  // fine histogram window around the predicted K-th value; outputs are
  // written when |v| > tw
  uint64_t win_lo, win_hi;
  double tw;
  gate_window(fin, gp, ctl, win_lo, win_hi, tw);

  for (int i = tid; i < kFineBins; i += BLOCK) sm.fhist[i] = 0;
  if (tid < kMaxClasses * kMaxClasses) sm.ncnt[tid] = 0;
  __shared__ Plan s_pin, s_pn;
  plan_to_lds(&s_pin, plan_in, tid);
  if constexpr (ADJ) plan_to_lds(&s_pn, adj.plan_next, tid - 128);
  __syncthreads();
  if (tid == 0) {
    const Plan* __restrict__ pin = &s_pin;
    uint64_t acc = 0;
    if constexpr (ADJ) {
      // the forward output, packed: region (c, e) holds exactly cnt[c][e]
      const Plan* __restrict__ pn = &s_pn;
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
  // tickets go out in arrival order, so the first total_tiles workgroups
  // can take them all: the others leave without touching the ticket counter
  // (for small states, hundreds of idle workgroups would otherwise queue on
  // that one atomic)
  if ((uint64_t)blockIdx.x >= total_tiles) return;
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
    // the reverse kernel reads the class views from LDS where it needs them
    // (kept in registers they make it spill); the forward kernel copies them
    using ViewT = std::conditional_t<ADJ, const ClassView&, const ClassView>;
    ViewT VA = sm.L.views[cA];
    ViewT VB = sm.L.views[cB];
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
      bool comm = !anticommutes(k, gp);
      if constexpr (RT) comm = !comm;  // the strings that branch
      // with a weight cutoff, the string's weight waits in rb[x] until the
      // walk reads it (the walk writes rb[x] only after that)
      if (gp.wmax) sm.rb[x] = (uint16_t)pauli_weight(k, gp.pos_in, nbits >> 1);
      if (!isA) k = xor_mask(k, gp.topm);  // B' = B xor Q lives in class cA's key space
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
            const Key<NW> ownk = isA ? k : xor_mask(k, gp.topm);
            bool neg = false;
            const uint32_t nph = (gp.lflags >> 6) & 7u;
            if (comm && nph) {
              const int e4 = (int)phase_e(ownk, gp.phpos, gp.etab, nph);
              if constexpr (RT) {
                // i Q P = i^(k+1) R: the own branch is -sin c for k = 1 and
                // +sin c for k = 3; the partner's branch (its phase is i^-k)
                // arrives with the opposite sign
                if (!(e4 & 1)) atomicMax(&ctl->error, kErrPhase);
                neg = (e4 == 3) != paired;
              } else {
                if (e4 & 1) atomicMax(&ctl->error, kErrPhase);
                neg = (e4 == 2);
              }
              if (neg) inf |= 512u;
            }
            T vs, vb;
            values_from<T>(c, comm, paired, cp, neg, ch, sh, vs, vb);
            bool hs = abs_d(vs) > tw;
            bool hb = comm && !paired && abs_d(vb) > tw;
            if (gp.wmax) {
              // weight cutoff (Sec. II.B): the self output keeps the
              // string's weight, the branch changes it on the support of Q
              const uint32_t wp = sm.rb[x];
              const uint32_t pat = support_pattern(ownk, gp.phpos, 2u * (uint32_t)gp.nsup);
              const uint32_t wr = wp + (uint32_t)((gp.wtab >> (3 * pat)) & 7u) - 2u;
              hs = hs && wp <= (uint32_t)gp.wmax;
              hb = hb && wr <= (uint32_t)gp.wmax;
            }
            if (paired) {
              inf |= 4u;
              sm.partner[x] = (uint16_t)y;
            }
            int es = (int)bit_at(ownk, (gp.fgpos >> 16) & 0xffu);
            if (gp.w1 > 1) es |= (int)bit_at(ownk, gp.fgpos >> 24) << 1;
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
      const unsigned long long tag32 = (unsigned long long)epoch << 32;
      const unsigned long long tag12 = (unsigned long long)(epoch % 4095u + 1u) << 52;
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
                  if ((x >> 32) == epoch) {
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
        uint32_t bb;
        Key<NW> mk = move_bit(k, gp.mvpos & 0xffu, (uint32_t)nbits - 1u, bb);
        if (gp.w1 > 1) mk = move_bit(mk, (gp.mvpos >> 8) & 0xffu, (uint32_t)nbits - 1u, bb);
        const Key<NW> ownk = x < nAt ? k : xor_mask(k, gp.topm);
        const uint32_t w2 = (gp.lflags >> 4) & 3u;
        int fself = 0;
        if (w2 > 0) fself = (int)bit_at(ownk, gp.fgpos & 0xffu);
        if (w2 > 1) fself |= (int)bit_at(ownk, (gp.fgpos >> 8) & 0xffu) << 1;
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
    uint64_t nb[4] = {0, 0, 0, 0};  // (next class, next-next class) counts, 16-bit fields
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
          bin_add(nb, es * kMaxClasses + fself);
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
          bin_add(nb, eb * kMaxClasses + (fself ^ gp.ovf));
        }
      }
    }
    if (written) atomicAdd(&sm.nwritten, written);
    if (above) atomicAdd(&sm.nabove, above);
    // the tile's class counts: one sum per wavefront, one LDS add per bin
    if (__ballot((nb[0] | nb[1] | nb[2] | nb[3]) != 0) != 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) nb[i] = wave_sum_u64(nb[i]);
      if (lane < kMaxClasses * kMaxClasses) {
        uint64_t v = nb[0];
#pragma unroll
        for (int i = 1; i < 4; ++i) v = ((lane >> 2) == i) ? nb[i] : v;
        const uint32_t cnt = (uint32_t)((v >> (16 * (lane & 3))) & 0xffffull);
        if (cnt) atomicAdd(&sm.ncnt[lane], cnt);
      }
    }
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
// Host launchers.
// Gate kernel shapes (threads per workgroup, merged elements per tile for
// one- and two-word keys).  Shape 0: one 1024-thread workgroup per CU with
// 4000/2000-string tiles; shape 1 (the default): two 512-thread workgroups
// per CU, each with the largest one-word tile whose LDS (about 32 B per
// string) still lets two share the CU's 160 KB, and 1500-string tiles for
// two-word keys.  Larger tiles pay the per-tile ticket, barriers and
// look-back less often.
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
    return NW == 2 ? 2380 : 1500;
  }
};

int gate_tile(int nw, int shape) {
  if (shape == 2) return layer_tile();
  if (shape == 1) return nw == 2 ? GateShape<1>::tile<2>() : GateShape<1>::tile<4>();
  return nw == 2 ? GateShape<0>::tile<2>() : GateShape<0>::tile<4>();
}
int gate_min_tile(int nw) { return std::min(std::min(gate_tile(nw, 0), gate_tile(nw, 1)), gate_tile(nw, 2)); }
int gate_wgs_per_cu(int shape) { return shape == 1 ? GateShape<1>::wgs_per_cu : GateShape<0>::wgs_per_cu; }

hipError_t launch_partition(int nw, const GateParams& gp, Side in, const Plan* plan_in, Ctl* ctl, uint64_t* part,
                            TileStatus* status, hipStream_t st) {
  // eight tile boundaries per wavefront, four wavefronts per block
  const uint64_t nb = gp.status_cap + kMaxClasses;
  const int pgrid = (int)((nb + 31) / 32);
  if (nw == 2)
    hipLaunchKernelGGL(partition_kernel<2>, dim3(pgrid), dim3(256), 0, st, gp, in, plan_in, part, ctl, status);
  else
    hipLaunchKernelGGL(partition_kernel<4>, dim3(pgrid), dim3(256), 0, st, gp, in, plan_in, part, ctl, status);
  return hipGetLastError();
}

template <int SHAPE, bool RT>
void launch_gate_shape(int nw, int f32, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                       Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part,
                       int grid, hipStream_t st) {
  using S = GateShape<SHAPE>;
  const AdjArgs none{};
  ITPP_DISPATCH(nw, f32,
                hipLaunchKernelGGL((gate_kernel<NWC, S::block, S::template tile<NWC>(), TC, false, RT>),
                                   dim3(grid), dim3(S::block), 0, st, gp, in, out, plan_in, plan_out, filt_in,
                                   (const uint64_t*)part, ctl, status, none));
}

hipError_t launch_gate(int nw, int f32, int shape, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                       Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part,
                       int grid, hipStream_t st) {
  if (shape == 1)
    launch_gate_shape<1, false>(nw, f32, gp, in, out, plan_in, plan_out, filt_in, ctl, status, part, grid, st);
  else
    launch_gate_shape<0, false>(nw, f32, gp, in, out, plan_in, plan_out, filt_in, ctl, status, part, grid, st);
  return hipGetLastError();
}

hipError_t launch_gate_rt(int nw, int f32, int shape, const GateParams& gp, Side in, Side out,
                          const Plan* plan_in, Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status,
                          uint64_t* part, int grid, hipStream_t st) {
  if (shape == 1)
    launch_gate_shape<1, true>(nw, f32, gp, in, out, plan_in, plan_out, filt_in, ctl, status, part, grid, st);
  else
    launch_gate_shape<0, true>(nw, f32, gp, in, out, plan_in, plan_out, filt_in, ctl, status, part, grid, st);
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

}  // namespace itpp
