// Selection, readout and bookkeeping kernels of the ITPP layer update
// (gfx950, wave64): the initial state rho = I, the exact top-K selection
// that decides the truncation after each gate (Sec. II.C, with the
// coefficient threshold of Sec. II.B), observables, export, and the
// packing, seeding and reduction kernels of the reverse sweep.
#include <hip/hip_runtime.h>

#include "itpp_device.h"
#include "itpp_readout.h"

namespace itpp {

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
  c.epoch = kStatusClearEvery;  // the first gate clears the look-back records
  *ctl = c;
}

// This lane's slot among the active lanes of its wave that pass `want`,
// reserved with one LDS atomic per wave on *counter.
__device__ __forceinline__ uint32_t wave_claim(bool want, uint32_t* counter) {
  const uint64_t act = __ballot(1);
  const uint64_t m = __ballot(want);
  const int lane = (int)(threadIdx.x & 63u);
  const int leader = __ffsll((unsigned long long)act) - 1;
  uint32_t base = 0;
  if (lane == leader && m) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = __shfl(base, leader, 64);
  return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Parallel search, over a histogram of nbins bins taken from the top,
// for the bin where the running count from above first reaches `need`
// (counts above the histogram: `base`).  Returns the bin (or -1) and the
// count above it; all threads must call.
__device__ inline void find_from_top(const uint32_t* h, int nbins, uint64_t base, uint64_t need,
                                     uint64_t* s_scratch, int* out_bin, uint64_t* out_above) {
  // blockDim.x is a multiple of 64 (every caller launches 256 or 1024 threads)
  const int tid = threadIdx.x;
  const int nth = blockDim.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int per = (nbins + nth - 1) / nth;
  // thread t owns bins nbins-1-t*per .. nbins-per-t*per (descending)
  uint64_t local = 0;
  for (int q = 0; q < per; ++q) {
    const int b = nbins - 1 - (tid * per + q);
    if (b >= 0) local += h[b];
  }
  // inclusive scan inside the wave, then the totals of the lower waves
  unsigned long long incl = local;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned long long v = __shfl_up(incl, d, 64);
    if (lane >= d) incl += v;
  }
  if (lane == 63) s_scratch[wv] = incl;
  __syncthreads();
  uint64_t wbase = 0;
  for (int q = 0; q < wv; ++q) wbase += s_scratch[q];
  uint64_t above = base + wbase + incl - local;
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
                                                      Ctl* ctl, int64_t K, int cap_fail, int spec, int spos) {
  __shared__ uint32_t fh[kFineBins];
  __shared__ uint64_t scr[1024];
  __shared__ int s_bin;
  __shared__ uint64_t s_above;
  const int tid = threadIdx.x;
  if (ctl->error || ctl->halt) return;
  // the decision the gate kernel took
  const bool specd = gate_speculates(*filt_in, spec, spos, ctl);
  {
    // a speculative gate that wrote fewer than K-1 strings above its write
    // threshold cannot decide the cap exactly: ask the host to redo it
    if (specd && (int64_t)ctl->n_written_nonid < K - 1) {
      __syncthreads();
      if (tid == 0) {
        ctl->halt = 1u;
        ctl->halt_serial = ctl->gate_serial;
        // the redone gate is a new attempt with a fresh look-back tag
        ctl->gate_serial += 1;
        ctl->epoch = next_epoch(ctl->epoch);
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
  // A speculative gate that stored exactly K strings stored the K largest
  // outputs (the ones it skipped are below its write threshold, hence below
  // every stored one): the cap binds at the smallest stored value.
  const bool capped = (int64_t)nw > K || (specd && (int64_t)nw == K);
  const uint64_t need = (uint64_t)(K - 1);
  uint64_t sel_lo = 0, sel_hi = 0, sel_need = 0;
  bool none_kept = false, coarse = false;
  if (capped && need == 0) {
    none_kept = true;
  } else if (capped) {
    // the window the gate kernel histogrammed (the same prediction)
    uint64_t win_lo = 0, win_hi = 0;
    const double pred = predicted_kth(fin, spos, ctl, nullptr);
    if (pred > 0.0) {
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
    ctl->written_elems += (double)nw;
    if (ctl->have_cI) {
      ctl->cI_min = cI < ctl->cI_min ? cI : ctl->cI_min;
      ctl->cI_max = cI > ctl->cI_max ? cI : ctl->cI_max;
    }
    ctl->alg_elems += (double)fin.n_survivors + (double)f.n_survivors;
    ctl->gates += 1;
    if (specd) ctl->spec_gates += 1;
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
    ctl->gate_serial += 1;
    ctl->epoch = next_epoch(ctl->epoch);
  }
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

// Canonical form of a rep key through the inverse bit map inv (rep position
// -> canonical bit, in LDS), visiting only the set bits: the strings of a tie
// group are mostly of low weight, so this is far cheaper than walking all
// 2n canonical bits.
template <int NW>
__device__ __forceinline__ Key<NW> canonical_sparse(const Key<NW>& k, const uint16_t* inv, int n) {
  constexpr int W = NW / 2;
  Key<NW> c;
#pragma unroll
  for (int i = 0; i < NW; ++i) c.w[i] = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    uint64_t w = k.w[i];
    while (w) {
      const int b = __ffsll((unsigned long long)w) - 1;
      w &= w - 1ull;
      const int cb = inv[64 * i + b];
      const int word = cb < n ? (cb >> 6) : (W + ((cb - n) >> 6));
      const int bit = cb < n ? (cb & 63) : ((cb - n) & 63);
      xor_bit(c, 64 * word + bit, 1ull);
    }
  }
  return c;
}

// Exact K-th value among the candidates (radix select on the |c| bits) and,
// for ties at that value, the largest canonical key still kept.
template <int NW>
__global__ __launch_bounds__(1024) void select_exact(Side out, const Filter* filt_in, Filter* filt_out, Ctl* ctl,
                                                     SelBuf sel, RepPos rp, int spos) {
  __shared__ uint32_t h[2048];
  __shared__ uint64_t scr[1024];
  __shared__ int s_bin;
  __shared__ uint64_t s_above;
  __shared__ uint32_t s_cnt0;
  __shared__ uint32_t s_ntie;
  // candidates left after the first radix pass, when few enough (bits, index)
  constexpr uint32_t kLdsCand = 4096;
  // tie sets up to this size are ranked directly (their keys fill lb)
  constexpr uint32_t kTieDirect = kLdsCand / kMaxKeyWords;
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
    // how far the K-th value moved from the raw prediction at this position
    double raw = 0.0;
    (void)predicted_kth(*filt_in, -1, ctl, &raw);
    if (spos >= 0 && raw > 0.0) ctl->kth_ratio[spos] = (float)(__longlong_as_double((long long)kth) / raw);
    const double kn = __longlong_as_double((long long)kth) / filt_out->cI;
    if (kn < ctl->kth_min) ctl->kth_min = kn;
  }
  __syncthreads();
  if (count_eq <= need_eq) return;
  // ties: gather canonical keys of the elements equal to kth
  __shared__ uint16_t inv[kMaxBits];
  for (int cb = tid; cb < rp.nbits; cb += blockDim.x) inv[rp.pos[cb]] = (uint16_t)cb;
  __syncthreads();
  const uint64_t mt = in_lds ? nl : m;
  for (uint64_t i = tid; i < mt; i += blockDim.x) {
    const bool tie = (in_lds ? lb[i] : sel.cand_bits[i]) == kth;
    // one LDS atomic per wave, not per tied element (tie groups can hold
    // hundreds of thousands of strings)
    const uint32_t slot = wave_claim(tie, &s_ntie);
    if (!tie) continue;
    Key<NW> k = load_key<NW>(out, sel.cand_idx[in_lds ? li[i] : i]);
    Key<NW> ck = canonical_sparse(k, inv, rp.nbits / 2);
    for (int q = 0; q < NW; ++q) sel.tie_keys[(uint64_t)slot * NW + q] = ck.w[q];
  }
  __syncthreads();
  const uint64_t nt = s_ntie;
  // The kept tied key is the needk-th smallest canonical key of the tied
  // keys matching (pre, msk) (they are distinct strings).  Once at most
  // kTieDirect keys match, they are ranked directly in LDS: the one with
  // exactly needk - 1 keys below it.
  uint64_t* tk = lb;  // the candidate list is no longer needed
  __shared__ uint32_t s_nd;
  auto rank_direct = [&](const uint64_t* keys, uint64_t nk, const Key<NW>& pre, const Key<NW>& msk,
                         uint64_t needk) {
    if (tid == 0) s_nd = 0;
    __syncthreads();
    for (uint64_t i = tid; i < nk; i += blockDim.x) {
      bool match = true;
      for (int q = 0; q < NW; ++q) match = match && ((keys[i * NW + q] & msk.w[q]) == pre.w[q]);
      const uint32_t slot = wave_claim(match, &s_nd);
      if (match)
        for (int q = 0; q < NW; ++q) tk[q * kTieDirect + slot] = keys[i * NW + q];
    }
    __syncthreads();
    const uint32_t nd = s_nd;
    for (uint32_t i = tid; i < nd; i += blockDim.x) {
      Key<NW> ki;
      for (int q = 0; q < NW; ++q) ki.w[q] = tk[q * kTieDirect + i];
      uint32_t below = 0;
      for (uint32_t j2 = 0; j2 < nd; ++j2) {
        Key<NW> kj;
        for (int q = 0; q < NW; ++q) kj.w[q] = tk[q * kTieDirect + j2];
        below += (j2 != i && canon_le(kj, ki)) ? 1u : 0u;
      }
      if ((uint64_t)below + 1u == needk) {
        filt_out->tie_active = 1;
        for (int q = 0; q < NW; ++q) filt_out->tie_key[q] = ki.w[q];
      }
    }
  };
  Key<NW> pre, msk;
  for (int q = 0; q < NW; ++q) pre.w[q] = msk.w[q] = 0;
  if (nt <= kTieDirect) {
    rank_direct(sel.tie_keys, nt, pre, msk, need_eq);
    return;
  }
  // the keys still matching the prefix, compacted after every pass into the
  // candidate arrays (free now), which hold sel.cap words each
  const uint64_t* keys = sel.tie_keys;
  uint64_t nk = nt;
  __shared__ uint32_t s_nc;
  // MSB-first radix selection (8-bit digits, X words before Z words) of
  // the need_eq-th smallest canonical key, until few enough keys match
  constexpr int W = NW / 2;
  const int n = rp.nbits / 2;
  const int ndig = (n + 7) / 8;  // digits per part; bits above n are zero in every key
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
      for (uint64_t i = tid; i < nk; i += blockDim.x) {
        bool match = true;
        for (int q = 0; q < NW; ++q) match = match && ((keys[i * NW + q] & msk.w[q]) == pre.w[q]);
        if (match) {
          atomicAdd(&h[(keys[i * NW + word] >> sh) & 0xffull], 1u);
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
      const uint32_t left = h[bsel];
      __syncthreads();
      if (left <= kTieDirect) {
        rank_direct(keys, nk, pre, msk, needk);
        return;
      }
      if ((uint64_t)left * NW <= sel.cap && left < nk) {
        uint64_t* dst = keys == sel.cand_bits ? sel.cand_idx : sel.cand_bits;
        if (tid == 0) s_nc = 0;
        __syncthreads();
        for (uint64_t i = tid; i < nk; i += blockDim.x) {
          bool match = true;
          for (int q = 0; q < NW; ++q) match = match && ((keys[i * NW + q] & msk.w[q]) == pre.w[q]);
          const uint32_t slot = wave_claim(match, &s_nc);
          if (match)
            for (int q = 0; q < NW; ++q) dst[(uint64_t)slot * NW + q] = keys[i * NW + q];
        }
        __syncthreads();
        keys = dst;
        nk = left;
      }
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
// Squared-state estimate (Sec. II.C): <O>_{2 tau} = Tr[(O rho) rho] / Tr[rho^2].
// With rho = 2^-n sum_P a_P P, every stored string P adds a_P^2 to the purity
// and, for each observable string Q_j it commutes with, o_j a_P a_R s to the
// numerator, where Q_j P = s R (s = +-1) and a_R is looked up in the stored
// state (anticommuting strings give imaginary terms that cancel in pairs).

// Normalised coefficient of key k in the stored state, if stored and kept.
template <int NW, typename T>
__device__ inline bool lookup_coef(const Side& s, const Plan& p, const Filter& f, const RepPos& rp,
                                   const Key<NW>& k, double& a) {
  const int e = class_of(k, rp.nbits, p.we);
  for (int c = 0; c < (1 << p.wc); ++c) {
    uint64_t lo = p.base[c][e], hi = p.base[c][e] + p.cnt[c][e];
    const uint64_t end = hi;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (key_less(load_key<NW>(s, mid), k))
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo < end && key_eq(load_key<NW>(s, lo), k)) {
      const T cs = coefs<T>(s)[lo];
      if (!survives(k, (double)cs, f, rp.pos, rp.nbits)) return false;
      a = (double)normalised<T>(cs, f.cI);
      return true;
    }
  }
  return false;
}

template <int NW, typename T>
__global__ __launch_bounds__(256) void squared_kernel(Side s, const Plan* plan, const Filter* filt, RepPos rp,
                                                      SqObs ob, Ctl* ctl, double* part) {
  __shared__ double red[4][256];
  const Plan& p = *plan;
  const Filter f = *filt;
  const int tid = threadIdx.x;
  double ns = 0.0, ne = 0.0, ps = 0.0, pe = 0.0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (int c = 0; c < (1 << p.wc); ++c)
    for (int e = 0; e < (1 << p.we); ++e) {
      const uint64_t base = p.base[c][e], cnt = p.cnt[c][e];
      for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + tid; i < cnt; i += stride) {
        const Key<NW> k = load_key<NW>(s, base + i);
        const T cs = coefs<T>(s)[base + i];
        if (!survives(k, (double)cs, f, rp.pos, rp.nbits)) continue;
        const double a = (double)normalised<T>(cs, f.cI);
        double sr, er;
        two_sum(ps, __dmul_rn(a, a), sr, er);
        ps = sr;
        pe = __dadd_rn(pe, er);
        for (int j = 0; j < ob.m; ++j) {
          int par = 0;
#pragma unroll
          for (int q = 0; q < NW; ++q) par ^= __popcll(k.w[q] & ob.cmask[(size_t)j * NW + q]) & 1;
          if (par) continue;
          Key<NW> r = k;
#pragma unroll
          for (int q = 0; q < NW; ++q) r.w[q] ^= ob.qmask[(size_t)j * NW + q];
          int e4 = ob.aq[j];
          for (int t = ob.sup_off[j]; t < ob.sup_off[j + 1]; ++t) {
            const int xp = get_bit(k, ob.sup_pos[2 * t]), zp = get_bit(k, ob.sup_pos[2 * t + 1]);
            const int qx = ob.sup_q[t] & 1, qz = (ob.sup_q[t] >> 1) & 1;
            e4 += (xp & zp) - ((xp ^ qx) & (zp ^ qz)) + 2 * (qz & xp);
          }
          e4 &= 3;
          if (e4 & 1) {
            atomicMax(&ctl->error, kErrPhase);
            continue;
          }
          double ar;
          if (!lookup_coef<NW, T>(s, p, f, rp, r, ar)) continue;
          double term = __dmul_rn(ob.coef[j], __dmul_rn(a, ar));
          if (e4 == 2) term = -term;
          two_sum(ns, term, sr, er);
          ns = sr;
          ne = __dadd_rn(ne, er);
        }
      }
    }
  red[0][tid] = ns;
  red[1][tid] = ne;
  red[2][tid] = ps;
  red[3][tid] = pe;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      double sr, er;
      two_sum(red[0][tid], red[0][tid + h], sr, er);
      red[0][tid] = sr;
      red[1][tid] = __dadd_rn(__dadd_rn(red[1][tid], red[1][tid + h]), er);
      two_sum(red[2][tid], red[2][tid + h], sr, er);
      red[2][tid] = sr;
      red[3][tid] = __dadd_rn(__dadd_rn(red[3][tid], red[3][tid + h]), er);
    }
    __syncthreads();
  }
  if (tid == 0) {
    part[4 * blockIdx.x + 0] = red[0][0];
    part[4 * blockIdx.x + 1] = red[1][0];
    part[4 * blockIdx.x + 2] = red[2][0];
    part[4 * blockIdx.x + 3] = red[3][0];
  }
}

// The per-block partials in a fixed order (one block of 256 threads).
__global__ __launch_bounds__(256) void squared_reduce(const double* part, int nparts, double* out) {
  __shared__ double red[4][256];
  const int tid = threadIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = tid; b < nparts; b += 256) {
    double sr, er;
    two_sum(v[0], part[4 * b + 0], sr, er);
    v[0] = sr;
    v[1] = __dadd_rn(__dadd_rn(v[1], part[4 * b + 1]), er);
    two_sum(v[2], part[4 * b + 2], sr, er);
    v[2] = sr;
    v[3] = __dadd_rn(__dadd_rn(v[3], part[4 * b + 3]), er);
  }
  for (int q = 0; q < 4; ++q) red[q][tid] = v[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      double sr, er;
      two_sum(red[0][tid], red[0][tid + h], sr, er);
      red[0][tid] = sr;
      red[1][tid] = __dadd_rn(__dadd_rn(red[1][tid], red[1][tid + h]), er);
      two_sum(red[2][tid], red[2][tid + h], sr, er);
      red[2][tid] = sr;
      red[3][tid] = __dadd_rn(__dadd_rn(red[3][tid], red[3][tid + h]), er);
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = __dadd_rn(red[0][0], red[1][0]);
    out[1] = __dadd_rn(red[2][0], red[3][0]);
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
    ctl->epoch = next_epoch(ctl->epoch);  // the reverse gate's look-back used this tag
  }
}

// ---------------------------------------------------------------------------
// Host launchers.

hipError_t launch_init(int nw, int f32, Side s0, Plan* plan, Filter* filt, Ctl* ctl, int w0, hipStream_t st) {
  ITPP_DISPATCH(nw, f32,
                hipLaunchKernelGGL((init_kernel<NWC, TC>), dim3(1), dim3(64), 0, st, s0, plan, filt, ctl, w0));
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
                         int64_t K, int cap_fail, int spec, int spos, int grid, hipStream_t st) {
  hipLaunchKernelGGL(select_decide, dim3(1), dim3(1024), 0, st, filt_in, filt_out, plan_next, ctl, K,
                     cap_fail, spec, spos);
  ITPP_DISPATCH(nw, f32, {
    hipLaunchKernelGGL((select_coarse_hist<NWC, TC>), dim3(grid / 4 > 0 ? grid / 4 : 1), dim3(256), 0, st, out,
                       plan_out, ctl);
    hipLaunchKernelGGL((select_collect<NWC, TC>), dim3(grid), dim3(256), 0, st, out, plan_out, ctl, sel);
    hipLaunchKernelGGL(select_exact<NWC>, dim3(1), dim3(1024), 0, st, out, filt_in, filt_out, ctl, sel, rp, spos);
  });
  return hipGetLastError();
}

// Observable tables of the squared-state readout, built on the device: per
// string j its flip mask (qmask), anticommutation mask (cmask) and support
// entries in ascending qubit order, exactly as the host-built tables.
__global__ __launch_bounds__(256) void sq_tables_kernel(RepPos rp, int n, int W, int NW, const uint64_t* x,
                                                        const uint64_t* z, const double* oc, int32_t m,
                                                        SqTables t) {
  const int tid = threadIdx.x;
  // support sizes, then their exclusive prefix (one thread: m is small)
  for (int j = tid; j < m; j += blockDim.x) {
    int cnt = 0;
    for (int q = 0; q < W; ++q) cnt += __popcll(x[(size_t)j * W + q] | z[(size_t)j * W + q]);
    t.sup_off[j + 1] = cnt;
  }
  __syncthreads();
  if (tid == 0) {
    t.sup_off[0] = 0;
    for (int j = 0; j < m; ++j) t.sup_off[j + 1] += t.sup_off[j];
  }
  __syncthreads();
  for (int j = tid; j < m; j += blockDim.x) {
    uint64_t qm[kMaxKeyWords] = {0, 0, 0, 0}, cm[kMaxKeyWords] = {0, 0, 0, 0};
    int e = t.sup_off[j], aq = 0;
    for (int i = 0; i < n; ++i) {
      const int xi = (int)((x[(size_t)j * W + (i >> 6)] >> (i & 63)) & 1ull);
      const int zi = (int)((z[(size_t)j * W + (i >> 6)] >> (i & 63)) & 1ull);
      if (!xi && !zi) continue;
      const int px = rp.pos[i], pz = rp.pos[n + i];
      if (xi) {
        qm[px >> 6] |= 1ull << (px & 63);
        cm[pz >> 6] |= 1ull << (pz & 63);  // x_Q z_P
      }
      if (zi) {
        qm[pz >> 6] |= 1ull << (pz & 63);
        cm[px >> 6] |= 1ull << (px & 63);  // z_Q x_P
      }
      t.sup_pos[2 * e] = px;
      t.sup_pos[2 * e + 1] = pz;
      t.sup_q[e] = xi | (zi << 1);
      aq += xi & zi;
      ++e;
    }
    for (int q = 0; q < NW; ++q) {
      t.qmask[(size_t)j * NW + q] = qm[q];
      t.cmask[(size_t)j * NW + q] = cm[q];
    }
    t.aq[j] = aq & 3;
    t.coef[j] = oc[j];
  }
}

hipError_t launch_sq_tables(const RepPos& rp, int n, int W, int NW, const uint64_t* x, const uint64_t* z,
                            const double* oc, int32_t m, SqTables t, hipStream_t st) {
  hipLaunchKernelGGL(sq_tables_kernel, dim3(1), dim3(256), 0, st, rp, n, W, NW, x, z, oc, m, t);
  return hipGetLastError();
}

hipError_t launch_squared(int nw, int f32, Side s, const Plan* plan, const Filter* filt, const RepPos& rp,
                          const SqObs& ob, Ctl* ctl, double* part, double* out, int grid, hipStream_t st) {
  ITPP_DISPATCH(nw, f32,
                hipLaunchKernelGGL((squared_kernel<NWC, TC>), dim3(grid), dim3(256), 0, st, s, plan, filt, rp, ob,
                                   ctl, part));
  hipLaunchKernelGGL(squared_reduce, dim3(1), dim3(256), 0, st, part, grid, out);
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
