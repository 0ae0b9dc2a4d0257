// The layer kernel: one elementary gate exp(-(theta/2) Q) of Algorithm 1
// (Eq. ITPP_PropRules) over the stored strings, for gfx950 (wave64).
//
// It computes exactly what gate_kernel computes (the same output regions,
// the same order inside them, the same statistics for the selection that
// follows) with a different shape:
//  * 256-thread workgroups on tiles of at most 1024 merged strings, several
//    workgroups per CU (5 for one-word keys, 3 for two-word keys), so that
//    while one workgroup waits in its look-back or at a barrier the others
//    compute and stream;
//  * a thread keeps the outputs of the strings it walks in registers (new
//    values computed once, keys moved into the next gate's bit order, their
//    classes and ranks) and writes them itself once the tile's region
//    offsets are known, so the tile's LDS holds only the loaded strings;
//  * the class-bit counts of this gate and of the next one are template
//    arguments, and every bit position the walk reads comes from per-gate
//    (word, shift) pairs and masks that the host precomputes;
//  * the per-output class counters of the next-next gate are counted in
//    registers and reduced per wavefront instead of by LDS atomics;
//  * the next tile's ticket and merge-path bounds are fetched while the
//    current tile is written.
// Pairing, merge-path tiles, the look-back and the deferred filter are as
// described in itpp_gate.hip.
#include <hip/hip_runtime.h>

#include "itpp_device.h"

namespace itpp {

namespace {

constexpr int kLayerBlock = 256;
constexpr int kLayerCapt = 1024;              // LDS slots per tile
constexpr int kLayerTile = kLayerCapt - 2;    // merged strings per tile (a moved pair adds one)
constexpr int kLayerPer = kLayerCapt / kLayerBlock;
constexpr int kLayerLB = 4;                   // look-back window: 64 * kLayerLB predecessors per round

template <int NW>
constexpr int layer_wgs_per_cu() {
  return NW == 2 ? 4 : 3;
}

template <int NW, typename T>
struct LayerSmem {
  uint64_t key[NW][kLayerCapt];  // A keys, then B keys xored into A's key space
  T coef[kLayerCapt];            // normalised input coefficients
  uint8_t info[kLayerCapt];      // bit0 survives the previous truncation, bit1 commutes (RT: branches)
  uint32_t meta[kLayerCapt];     // per merged position: outputs, classes, ranks (see layer_kernel)
  uint32_t xy[kLayerCapt];       // per merged position: the string's slot and its partner's
  uint32_t fhist[kFineBins];
  uint32_t ncnt[kMaxClasses * kMaxClasses];
  uint64_t out_base[kMaxClasses + 1][kMaxClasses];  // row kMaxClasses holds the total
  uint64_t wa[kLayerBlock / 64], wb[kLayerBlock / 64];
  uint64_t tot0, tot1;
  uint32_t excl[2 * kMaxClasses];
  uint64_t pf[4];
  uint64_t abase, bbase;  // physical position of the tile's first A / B string
  uint32_t contig;        // 1: each of the two ranges lies in one region
  uint32_t tile;
  uint32_t nwritten, nabove;
  JoinLayout L;
};


// Look-back across the tiles of one join (wave 0): the exclusive prefix of
// the 8 region counters (stream cA / cB x next class) of tile t, from the
// predecessors' aggregates and the nearest published inclusive prefix.
// Record format as in gate_kernel: two self-validating aggregate words per
// tile (12-bit counts, 12-bit epoch tag, bit 48 = inclusive published) and
// one inclusive word per counter ((epoch << 32) | count).  Every word
// carries its epoch, and a reader spins on the inclusive word itself until
// its epoch matches, so bit 48 is only a hint and no fence orders the
// stores (an agent-scope release fence writes back the whole L2 of the XCD).
__device__ inline void layer_lookback(TileStatus* __restrict__ status, uint64_t SN, uint64_t t, bool first_tile,
                                      int64_t first, uint32_t epoch, uint64_t tot0, uint64_t tot1, Ctl* ctl,
                                      uint32_t (&excl)[2 * kMaxClasses]) {
  constexpr int NQ = 2 * kMaxClasses;
  const int lane = threadIdx.x & 63;
  uint32_t agg[NQ];
#pragma unroll
  for (int e = 0; e < kMaxClasses; ++e) {
    agg[e] = lane16(tot0, e);
    agg[kMaxClasses + e] = lane16(tot1, e);
  }
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
#pragma unroll
  for (int q = 0; q < NQ; ++q) excl[q] = 0;
  if (first_tile) {
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < NQ; ++q)
        __hip_atomic_store(&status[(2 + q) * SN + t], tag32 | agg[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int sd = 0; sd < 2; ++sd)
        __hip_atomic_store(&status[sd * SN + t], aw[sd] | kInclReady, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  if (lane == 0) {
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
      __hip_atomic_store(&status[sd * SN + t], aw[sd], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  constexpr int LB = kLayerLB;
  int64_t khi = (int64_t)t - 1;
  bool done = false;
  while (!done) {
    unsigned long long w0[LB], w1[LB];
    uint32_t pend = 0;  // this lane's slots not yet published (per lane: only those are polled again)
#pragma unroll
    for (int r = 0; r < LB; ++r) {
      w0[r] = kInclReady;  // before the join's first tile: ready with zero counts
      w1[r] = 0;
      if (khi - (int64_t)(r * 64 + lane) >= first) pend |= 1u << r;
    }
    uint32_t spins = 0;
    while (__ballot(pend != 0) != 0) {
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
      if (__ballot(pend != 0) == 0) break;
      if (++spins > (1u << 20)) {
        atomicMax(&ctl->error, kErrSpin);
#pragma unroll
        for (int r = 0; r < LB; ++r)
          if ((pend >> r) & 1u) {
            w0[r] = kInclReady;
            w1[r] = 0;
          }
        pend = 0;
        break;
      }
      // back off: a predecessor still loading or walking takes microseconds
      if (spins < 4)
        __builtin_amdgcn_s_sleep(2);
      else
        __builtin_amdgcn_s_sleep(16);
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
          uint32_t sp = 0;
          for (;;) {
            const unsigned long long x =
                __hip_atomic_load(&status[(2 + lane) * SN + kp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((x >> 32) == epoch) {
              iv = (uint32_t)x;
              break;
            }
            if (++sp > (1u << 20)) {
              atomicMax(&ctl->error, kErrSpin);
              break;
            }
            if (sp < 4)
              __builtin_amdgcn_s_sleep(2);
            else
              __builtin_amdgcn_s_sleep(16);
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

// Ticket and merge-path bounds of the next tile, with the physical
// position of its first A and first B string when each range lies inside
// one region of the input (contig; almost always, regions are long).
__device__ __forceinline__ void fetch_tile(const JoinLayout& L, const uint64_t* __restrict__ part, Ctl* ctl,
                                           int full, uint32_t& t, uint64_t pf[4], uint64_t& abase, uint64_t& bbase,
                                           uint32_t& contig);

// Segment (region) of element i of a class view.
__device__ __forceinline__ int view_seg(const ClassView& v, uint64_t i) {
  int sg = 0;
#pragma unroll
  for (int t = 1; t < kMaxClasses; ++t)
    if (t < v.nseg && i >= v.start[t]) sg = t;
  return sg;
}

__device__ __forceinline__ uint64_t view_phys(const ClassView& v, uint64_t i) {
  uint64_t b = v.base[0], st = 0;
#pragma unroll
  for (int t = 1; t < kMaxClasses; ++t) {
    const bool in = (t < v.nseg) && (i >= v.start[t]);
    b = in ? v.base[t] : b;
    st = in ? v.start[t] : st;
  }
  return b + (i - st);
}

__device__ __forceinline__ void fetch_tile(const JoinLayout& L, const uint64_t* __restrict__ part, Ctl* ctl,
                                           int full, uint32_t& t, uint64_t pf[4], uint64_t& abase, uint64_t& bbase,
                                           uint32_t& contig) {
  t = atomicAdd(&ctl->ticket, 1u);
  const uint64_t total = L.tiles_before[L.njoin];
  pf[0] = pf[1] = pf[2] = pf[3] = 0;
  abase = bbase = 0;
  contig = 1;
  if (t < total) {
    int j = 0;
    while (j + 1 < L.njoin && t >= L.tiles_before[j + 1]) ++j;
    const uint64_t pb = L.tiles_before[j] + (uint64_t)j + (t - L.tiles_before[j]);
#pragma unroll
    for (int q = 0; q < 4; ++q) pf[q] = part[2 * pb + q];
    const ClassView& VA = L.views[j];
    const ClassView& VB = L.views[j ^ full];
    if (pf[2] > pf[0]) {
      abase = view_phys(VA, pf[0]);
      if (view_seg(VA, pf[0]) != view_seg(VA, pf[2] - 1)) contig = 0;
    }
    if (pf[3] > pf[1]) {
      bbase = view_phys(VB, pf[1]);
      if (view_seg(VB, pf[1]) != view_seg(VB, pf[3] - 1)) contig = 0;
    }
  }
}

template <int NW>
__device__ __forceinline__ Key<NW> lkey(const uint64_t (*key)[kLayerCapt], int x) {
  Key<NW> k;
#pragma unroll
  for (int q = 0; q < NW; ++q) k.w[q] = key[q][x];
  return k;
}

// New values of a string (Eq. ITPP_PropRules; for an unpaired commuting
// string also its branch QP); neg: Q P = -R.
template <typename T>
__device__ __forceinline__ void new_values(T c, bool comm, bool paired, T cp, bool neg, T ch, T sh, T& vs, T& vb) {
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


// Per walked string, kept in registers from the walk to the write:
// meta: bit0 self output, bit1 branch output, bit2 the string is in class
// cA, bits 3-4 / 5-6 class of the self / branch output under the next gate,
// bits 7-8 the self output's class under the gate after next, bits 9-11 /
// 12-14 rank of the self / branch output in the thread's run, bit 15 Q P =
// -R, bit 16 commuting (RT: branching), bit 17 paired; xy: the string's
// slot and its partner's.
template <int NW, typename T, bool RT, int WC, int WN>
__global__ __launch_bounds__(kLayerBlock) __attribute__((amdgpu_waves_per_eu(layer_wgs_per_cu<NW>())))
void layer_kernel(GateParams gp, Side in, Side out, const Plan* __restrict__ plan_in, Plan* __restrict__ plan_out,
                  const Filter* __restrict__ filt_in, const uint64_t* __restrict__ part, Ctl* __restrict__ ctl,
                  TileStatus* __restrict__ status) {
  using Smem = LayerSmem<NW, T>;
  constexpr int BLOCK = kLayerBlock, PER = kLayerPer;
  constexpr int ncls = 1 << WC, full = ncls - 1, ncls1 = 1 << WN;
  __shared__ Smem sm;
  const int tid = threadIdx.x;
  if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kErrNone || ctl->halt) return;
  const double cI = filt_in->cI;
  const uint32_t epoch = ctl->epoch;
  const uint64_t kth_bits = filt_in->kth_bits;
  const bool cap_active = filt_in->cap_active != 0;
  const bool tie_active = filt_in->tie_active != 0;
  const T ch = (T)gp.ch, sh = (T)gp.sh;
  const uint32_t nbits = (uint32_t)gp.nbits, top = nbits - 1u;
  // fine histogram window around the predicted K-th value; outputs are
  // written when |v| > tw
  uint64_t win_lo, win_hi;
  double tw;
  gate_window(*filt_in, gp, ctl, win_lo, win_hi, tw);
  for (int i = tid; i < kFineBins; i += BLOCK) sm.fhist[i] = 0;
  if (tid < kMaxClasses * kMaxClasses) sm.ncnt[tid] = 0;
  __shared__ Plan s_pin;
  plan_to_lds(&s_pin, plan_in, tid);
  __syncthreads();
  if (tid == 0) {
    const Plan* __restrict__ pin = &s_pin;
    const int ov = (int)(gp.lflags & 3u);
    // output region capacities: cap(c, e) = n[c][e] + n[~c][e ^ ov]
    uint64_t acc = 0;
    for (int c = 0; c < kMaxClasses; ++c)
      for (int e = 0; e < kMaxClasses; ++e) {
        sm.out_base[c][e] = acc;
        if (c < ncls && e < ncls1) acc += (uint64_t)pin->ncnt[c][e] + (uint64_t)pin->ncnt[c ^ full][e ^ ov];
      }
    for (int e = 0; e < kMaxClasses; ++e) sm.out_base[kMaxClasses][e] = acc;
    if (acc > gp.cap_elems) atomicMax(&ctl->error, kErrCapacity);
    if (blockIdx.x == 0) {
      for (int c = 0; c < kMaxClasses; ++c)
        for (int e = 0; e < kMaxClasses; ++e) plan_out->base[c][e] = sm.out_base[c][e];
      plan_out->wc = WC;
      plan_out->we = WN;
    }
    sm.nwritten = 0;
    sm.nabove = 0;
    make_layout(sm.L, pin, WC, kLayerTile);
  }
  __syncthreads();
  const uint64_t total_tiles = sm.L.tiles_before[sm.L.njoin];
  if (__hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != kErrNone || ctl->halt) return;
  // the first total_tiles workgroups can take every ticket (arrival order)
  if ((uint64_t)blockIdx.x >= total_tiles) return;
  if (tid == 0) {
    uint32_t t0, ct;
    uint64_t pf[4], ab, bb;
    fetch_tile(sm.L, part, ctl, full, t0, pf, ab, bb, ct);
    sm.tile = t0;
#pragma unroll
    for (int q = 0; q < 4; ++q) sm.pf[q] = pf[q];
    sm.abase = ab;
    sm.bbase = bb;
    sm.contig = ct;
  }
  __syncthreads();

  uint32_t written = 0, above = 0;
  for (;;) {
    const uint64_t t = sm.tile;
    if (t >= total_tiles) break;
    if (t >= gp.status_cap) {
      if (tid == 0) atomicMax(&ctl->error, kErrCapacity);
      break;
    }
    int j = 0;
    while (j + 1 < sm.L.njoin && t >= sm.L.tiles_before[j + 1]) ++j;
    const uint64_t first = sm.L.tiles_before[j];
    const int cA = j, cB = j ^ full;
    const uint64_t i0 = sm.pf[0], j0 = sm.pf[1];
    const int nAt = (int)(sm.pf[2] - i0);
    const int nBt = (int)(sm.pf[3] - j0);
    const int nt = nAt + nBt;
    if (nt > kLayerCapt || nAt < 0 || nBt < 0) {
      if (tid == 0) atomicMax(&ctl->error, kErrCapacity);
      break;
    }

    // (1) load with the previous gate's filter and normalisation
    {
      const bool contig = sm.contig != 0;
      const uint64_t abase = sm.abase, bbase = sm.bbase;
      Key<NW> lk[PER];
      T lc[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int x = tid + q * BLOCK;
        if (x < nt) {
          uint64_t p;
          if (contig)
            p = x < nAt ? abase + (uint64_t)x : bbase + (uint64_t)(x - nAt);
          else
            p = x < nAt ? view_phys(sm.L.views[cA], i0 + x) : view_phys(sm.L.views[cB], j0 + (x - nAt));
          lk[q] = load_key<NW>(in, p);
          lc[q] = coefs<T>(in)[p];
        }
      }
      bool ties = false;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int x = tid + q * BLOCK;
        if (x < nt) {
          Key<NW> k = lk[q];
          const T cs = lc[q];
          // bit 2: |c| equals the K-th value, decided by the tie-break below
          uint32_t sv = 1u;
          if (cap_active && !key_zero(k)) {
            const uint64_t b = abs_bits((double)cs);
            sv = b > kth_bits ? 1u : 0u;
            if (b == kth_bits) sv = tie_active ? 4u : 1u;
          }
          ties = ties || sv == 4u;
          bool comm = !anticommutes(k, gp);
          if constexpr (RT) comm = !comm;  // the strings that branch
          if (x >= nAt) {
            // B' = B xor Q lives in class cA's key space (Q flips the top WC bits)
            flip_at(k, top);
            if constexpr (WC == 2) flip_at(k, top - 1u);
          }
#pragma unroll
          for (int w = 0; w < NW; ++w) sm.key[w][x] = k.w[w];
          sm.coef[x] = normalised<T>(cs, cI);
          sm.info[x] = (uint8_t)(sv | (comm ? 2u : 0u));
        }
      }
      // tie-break of the previous truncation: a string whose |c| equals the
      // K-th value survives when its canonical key is at most the last kept
      if (ties) {
        Key<NW> tk;
#pragma unroll
        for (int w = 0; w < NW; ++w) tk.w[w] = filt_in->tie_key[w];
#pragma unroll 1
        for (int q = 0; q < PER; ++q) {
          const int x = tid + q * BLOCK;
          if (x < nt && (sm.info[x] & 4u)) {
            Key<NW> k = lkey<NW>(sm.key, x);
            if (x >= nAt) {
              flip_at(k, top);
              if constexpr (WC == 2) flip_at(k, top - 1u);
            }
            const bool keep = canon_le(to_canonical(k, gp.pos_in, (int)nbits), tk);
            sm.info[x] = (uint8_t)((sm.info[x] & 2u) | (keep ? 1u : 0u));
          }
        }
      }
    }
    __syncthreads();

    // (2) merge walk over merged positions [m0, m0 + PER): A before B on
    // equal keys, an equal B follows its A partner
    uint64_t c0 = 0, c1 = 0;  // run counts per next class (16-bit lanes): stream cA, stream cB
    const int m0 = tid * PER;
    const int m1 = (m0 + PER < nt) ? m0 + PER : nt;
    {
      const uint32_t lf = gp.lflags;
      int a = 0, b = 0;
      Key<NW> kprev;  // the A string before position a (partner of an equal B)
#pragma unroll
      for (int w = 0; w < NW; ++w) kprev.w[w] = 0;
      bool have_prev = false;
      if (m0 < nt) {
        int lo = m0 > nBt ? m0 - nBt : 0;
        int hi = m0 < nAt ? m0 : nAt;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          const Key<NW> ka = lkey<NW>(sm.key, mid);
          const Key<NW> kb = lkey<NW>(sm.key, nAt + (m0 - mid - 1));
          if (!key_less(kb, ka))
            lo = mid + 1;
          else
            hi = mid;
        }
        a = lo;
        b = m0 - lo;
        if (a > 0) {
          kprev = lkey<NW>(sm.key, a - 1);
          have_prev = true;
        }
      }
#pragma unroll 1
      for (int m = m0; m < m1; ++m) {
        {
          const bool haveA = a < nAt, haveB = b < nBt;
          Key<NW> ka, kb;
#pragma unroll
          for (int w = 0; w < NW; ++w) ka.w[w] = kb.w[w] = 0;
          if (haveA) ka = lkey<NW>(sm.key, a);
          if (haveB) kb = lkey<NW>(sm.key, nAt + b);
          const bool isA = haveA && (!haveB || !key_less(kb, ka));
          const int x = isA ? a : nAt + b;
          int y = -1;
          if (isA) {
            if (haveB && key_eq(ka, kb)) y = nAt + b;
          } else if (have_prev && key_eq(kprev, kb)) {
            y = a - 1;
          }
          const Key<NW> k = isA ? ka : kb;
          const uint32_t inf = sm.info[x];
          uint32_t mt = 0;
          if (inf & 1u) {
            const bool comm = (inf >> 1) & 1u;
            const bool paired = (y >= 0) && (sm.info[y] & 1u);
            const T c = sm.coef[x];
            const T cp = paired ? sm.coef[y] : (T)0;
            bool neg = false;
            const uint32_t nph = (lf >> 6) & 7u;
            if (comm && nph) {
              const uint32_t pp = gp.phpos;
              uint32_t idx = bit_at(k, pp & 0xffu) | (bit_at(k, (pp >> 8) & 0xffu) << 1);
              if (nph > 2) idx |= (bit_at(k, (pp >> 16) & 0xffu) << 2) | (bit_at(k, pp >> 24) << 3);
              if (!isA) idx ^= (lf >> 9) & 15u;  // the phase is that of the string's own key
              const uint32_t e4 = (gp.etab >> (2 * idx)) & 3u;
              if constexpr (RT) {
                // i Q P = i^(k+1) R: the own branch is -sin c for k = 1 and
                // +sin c for k = 3; the partner's branch (its phase is i^-k)
                // arrives with the opposite sign
                if (!(e4 & 1u)) atomicMax(&ctl->error, kErrPhase);
                neg = (e4 == 3u) != paired;
              } else {
                if (e4 & 1u) atomicMax(&ctl->error, kErrPhase);
                neg = e4 == 2u;
              }
            }
            T v0, v1;
            new_values<T>(c, comm, paired, cp, neg, ch, sh, v0, v1);
            const bool hs = abs_d(v0) > tw;
            const bool hb = comm && !paired && abs_d(v1) > tw;
            if (hs || hb) {
              // classes under the next gate and the gate after next, read
              // from k (the own key is k for an A string, k xor Q for B)
              const uint32_t fg = gp.fgpos;
              uint32_t ek = bit_at(k, (fg >> 16) & 0xffu);
              if constexpr (WN == 2) ek |= bit_at(k, fg >> 24) << 1;
              const uint32_t w2 = (lf >> 4) & 3u;
              uint32_t fk = 0;
              if (w2 > 0) fk = bit_at(k, fg & 0xffu);
              if (w2 > 1) fk |= bit_at(k, (fg >> 8) & 0xffu) << 1;
              const uint32_t ov = lf & 3u, ovf = (lf >> 2) & 3u;
              const uint32_t es = isA ? ek : (ek ^ ov);
              const uint32_t eb = es ^ ov;
              const uint32_t fs = isA ? fk : (fk ^ ovf);
              mt = (hs ? 1u : 0u) | (hb ? 2u : 0u) | (isA ? 4u : 0u) | (es << 3) | (eb << 5) | (fs << 7) |
                   (neg ? (1u << 15) : 0u) | (comm ? (1u << 16) : 0u) | (paired ? (1u << 17) : 0u);
              // A: self -> stream cA, branch -> stream cB; B: the reverse
              if (hs) {
                const uint64_t cs = isA ? c0 : c1;
                mt |= (uint32_t)lane16(cs, (int)es) << 9;
                const uint64_t inc = 1ull << (16 * es);
                if (isA)
                  c0 += inc;
                else
                  c1 += inc;
              }
              if (hb) {
                const uint64_t cb = isA ? c1 : c0;
                mt |= (uint32_t)lane16(cb, (int)eb) << 12;
                const uint64_t inc = 1ull << (16 * eb);
                if (isA)
                  c1 += inc;
                else
                  c0 += inc;
              }
              sm.xy[m] = (uint32_t)x | ((uint32_t)(y < 0 ? 0 : y) << 16);
            }
          }
          sm.meta[m] = mt;
          if (isA) {
            kprev = ka;
            have_prev = true;
            ++a;
          } else {
            ++b;
          }
        }
      }
    }
    // (3) block scan of the run counts: thread prefixes inside the tile
    uint64_t p0 = c0, p1 = c1;
    {
      uint64_t t0, t1;
      block_scan2<BLOCK>(p0, p1, sm.wa, sm.wb, t0, t1);
      if (tid == 0) {
        sm.tot0 = t0;
        sm.tot1 = t1;
      }
    }
    __syncthreads();
    // (4) look-back across the tiles of this join (wave 0)
    if (tid < 64) {
      uint32_t excl[2 * kMaxClasses];
      layer_lookback(status, gp.status_cap, t, t == first, (int64_t)first, epoch, sm.tot0, sm.tot1, ctl, excl);
      if (tid == 0) {
#pragma unroll
        for (int q = 0; q < 2 * kMaxClasses; ++q) sm.excl[q] = excl[q];
        // the last tile of the join publishes the region fill counts
        if (t + 1 == sm.L.tiles_before[j + 1]) {
#pragma unroll
          for (int e = 0; e < kMaxClasses; ++e) {
            if (e < ncls1) {
              plan_out->cnt[cA][e] = excl[e] + lane16(sm.tot0, e);
              plan_out->cnt[cB][e] = excl[kMaxClasses + e] + lane16(sm.tot1, e);
            }
          }
        }
      }
    }
    __syncthreads();
    // the next tile's ticket and bounds, fetched while this one is written.
    // Tickets are taken once a tile's look-back is done, so tiles start in
    // about ticket order and a look-back finds its predecessors started.
    if (tid == 64) {
      uint32_t tn, ct;
      uint64_t pf[4], ab, bb;
      fetch_tile(sm.L, part, ctl, full, tn, pf, ab, bb, ct);
      sm.tile = tn;
#pragma unroll
      for (int q = 0; q < 4; ++q) sm.pf[q] = pf[q];
      sm.abase = ab;
      sm.bbase = bb;
      sm.contig = ct;
    }
    // (5) write: values and keys in the next gate's bit order, recomputed
    // from the tile still in LDS
    uint64_t nb[4] = {0, 0, 0, 0};
    {
      const uint32_t lf = gp.lflags;
      const uint32_t ovf = (lf >> 2) & 3u;
#pragma unroll 1
      for (int mp = m0; mp < m1; ++mp) {
        const uint32_t mt = sm.meta[mp];
        if (!(mt & 3u)) continue;
        const uint32_t xyv = sm.xy[mp];
        const int x = (int)(xyv & 0xffffu), y = (int)(xyv >> 16);
        const bool isA = (mt >> 2) & 1u;
        const int es = (mt >> 3) & 3, eb = (mt >> 5) & 3, fs = (mt >> 7) & 3;
        const bool paired = (mt >> 17) & 1u;
        T v0, v1;
        new_values<T>(sm.coef[x], (mt >> 16) & 1u, paired, paired ? sm.coef[y] : (T)0, (mt >> 15) & 1u, ch, sh, v0,
                      v1);
        uint32_t bb;
        Key<NW> m = move_bit(lkey<NW>(sm.key, x), gp.mvpos & 0xffu, top, bb);
        if constexpr (WN == 2) m = move_bit(m, (gp.mvpos >> 8) & 0xffu, top, bb);
        Key<NW> mq = m;  // the key of the other output: this gate's bits flipped
        flip_at(mq, gp.q1pos & 0xffu);
        if constexpr (WC == 2) flip_at(mq, (gp.q1pos >> 8) & 0xffu);
        if (mt & 1u) {
          const int stream = isA ? 0 : 1;
          const int cls = isA ? cA : cB;
          const uint64_t pos = sm.out_base[cls][es] + sm.excl[stream * kMaxClasses + es] +
                               lane16(isA ? p0 : p1, es) + ((mt >> 9) & 7u);
          const Key<NW> ks = isA ? m : mq;
          if (pos >= region_end(sm.out_base, cls, es)) {
            atomicMax(&ctl->error, kErrCapacity);
          } else {
            store_key<NW>(out, pos, ks);
            coefs<T>(out)[pos] = v0;
            if (key_zero(ks)) {
              ctl->cI_out = (double)v0;
              ctl->have_cI = 1u;
            } else {
              const uint64_t bits = abs_bits((double)v0);
              if (bits >= win_hi)
                ++above;
              else if (bits >= win_lo)
                atomicAdd(&sm.fhist[(bits - win_lo) >> kFineShift], 1u);
              ++written;
            }
            bin_add(nb, es * kMaxClasses + fs);
          }
        }
        if (mt & 2u) {
          const int stream = isA ? 1 : 0;
          const int cls = isA ? cB : cA;
          const uint64_t pos = sm.out_base[cls][eb] + sm.excl[stream * kMaxClasses + eb] +
                               lane16(isA ? p1 : p0, eb) + ((mt >> 12) & 7u);
          const Key<NW> kb = isA ? mq : m;
          if (pos >= region_end(sm.out_base, cls, eb)) {
            atomicMax(&ctl->error, kErrCapacity);
          } else {
            store_key<NW>(out, pos, kb);
            coefs<T>(out)[pos] = v1;
            const uint64_t bits = abs_bits((double)v1);
            if (bits >= win_hi)
              ++above;
            else if (bits >= win_lo)
              atomicAdd(&sm.fhist[(bits - win_lo) >> kFineShift], 1u);
            ++written;
            bin_add(nb, eb * kMaxClasses + (int)((uint32_t)fs ^ ovf));
          }
        }
      }
    }
    // (6) the tile's (class, next-next class) counts: one sum per wavefront
    {
      const uint64_t any = nb[0] | nb[1] | nb[2] | nb[3];
      if (__ballot(any != 0) != 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) nb[i] = wave_sum_u64(nb[i]);
        const int lane = tid & 63;
        if (lane < kMaxClasses * kMaxClasses) {
          uint64_t v = nb[0];
#pragma unroll
          for (int i = 1; i < 4; ++i) v = ((lane >> 2) == i) ? nb[i] : v;
          const uint32_t cnt = (uint32_t)((v >> (16 * (lane & 3))) & 0xffffull);
          if (cnt) atomicAdd(&sm.ncnt[lane], cnt);
        }
      }
    }
    // the next tile's load overwrites the tile every thread has just read
    __syncthreads();
  }
  // flush per-workgroup statistics
  {
    const uint64_t wv = wave_sum_u64(((uint64_t)above << 32) | written);
    if ((tid & 63) == 0 && wv) {
      atomicAdd(&sm.nwritten, (uint32_t)wv);
      atomicAdd(&sm.nabove, (uint32_t)(wv >> 32));
    }
  }
  __syncthreads();
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

template <int NW, typename T, bool RT>
void launch_layer_nw(const GateParams& gp, Side in, Side out, const Plan* plan_in, Plan* plan_out,
                     const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part, int cus, hipStream_t st) {
  const int grid = cus * layer_wgs_per_cu<NW>();
  const uint64_t* pt = part;
#define ITPP_LAYER(WC_, WN_)                                                                                      \
  hipLaunchKernelGGL((layer_kernel<NW, T, RT, WC_, WN_>), dim3(grid), dim3(kLayerBlock), 0, st, gp, in, out, \
                     plan_in, plan_out, filt_in, pt, ctl, status)
  if (gp.w == 1 && gp.w1 == 1)
    ITPP_LAYER(1, 1);
  else if (gp.w == 1)
    ITPP_LAYER(1, 2);
  else if (gp.w1 == 1)
    ITPP_LAYER(2, 1);
  else
    ITPP_LAYER(2, 2);
#undef ITPP_LAYER
}

}  // namespace

int layer_tile() { return kLayerTile; }

hipError_t launch_layer(int nw, int f32, bool rt, const GateParams& gp, Side in, Side out, const Plan* plan_in,
                        Plan* plan_out, const Filter* filt_in, Ctl* ctl, TileStatus* status, uint64_t* part, int cus,
                        hipStream_t st) {
  if (gp.w < 1 || gp.w > 2 || gp.w1 < 1 || gp.w1 > 2) return hipErrorInvalidValue;
  if (rt) {
    ITPP_DISPATCH(nw, f32,
                  (launch_layer_nw<NWC, TC, true>(gp, in, out, plan_in, plan_out, filt_in, ctl, status, part, cus, st)));
  } else {
    ITPP_DISPATCH(nw, f32,
                  (launch_layer_nw<NWC, TC, false>(gp, in, out, plan_in, plan_out, filt_in, ctl, status, part, cus,
                                                  st)));
  }
  return hipGetLastError();
}

}  // namespace itpp
