// Readout of the squared-state estimate (Sec. II.C, <O>_{2 tau}): device
// description of the observable strings and the launcher.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "itpp_internal.h"

namespace itpp {

// Observable strings in rep coordinates (device arrays).  String j flips the
// rep bits qmask[j*NW .. j*NW + NW) and anticommutes with a stored string when
// that string's bits under cmask[j*NW ..] have odd parity.  Its non-identity
// sites are t in [sup_off[j], sup_off[j+1]): rep positions sup_pos[2t] (x bit)
// and sup_pos[2t+1] (z bit), letter bits sup_q[t] (bit 0 x, bit 1 z).
// aq[j] is its number of Y letters mod 4, coef[j] its weight o_j.
struct SqObs {
  int32_t m;
  const uint64_t* qmask;
  const uint64_t* cmask;
  const int32_t* sup_off;
  const int32_t* sup_pos;
  const int32_t* sup_q;
  const int32_t* aq;
  const double* coef;
};

// Writable view of the same arrays, filled on the device by
// launch_sq_tables from canonical observable words.
struct SqTables {
  uint64_t* qmask;
  uint64_t* cmask;
  int32_t* sup_off;
  int32_t* sup_pos;
  int32_t* sup_q;
  int32_t* aq;
  double* coef;
};

// Builds the tables of m observable strings (canonical words: W x words then
// W z words per string at x + j*W, z + j*W; weights oc) for a stored state
// whose canonical bit b sits at rep position rp.pos[b] (one workgroup; the
// support entries of string j start at the sum of the supports before it).
hipError_t launch_sq_tables(const RepPos& rp, int n, int W, int NW, const uint64_t* x, const uint64_t* z,
                            const double* oc, int32_t m, SqTables t, hipStream_t st);

// part: 4 doubles per block of the first kernel (numerator and purity, each
// with its compensation); out: numerator and purity.
hipError_t launch_squared(int nw, int f32, Side s, const Plan* plan, const Filter* filt, const RepPos& rp,
                          const SqObs& ob, Ctl* ctl, double* part, double* out, int grid, hipStream_t st);

}  // namespace itpp
