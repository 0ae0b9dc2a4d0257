/*
 * itpp.h -- C ABI of the MI355X (gfx950) imaginary-time Pauli propagation
 * engine (arXiv 2601.14400, "Pauli Propagation for Imaginary-Time Evolution").
 *
 * The engine keeps a density matrix rho = 2^-n sum_P a_P P as a sparse set of
 * Pauli strings with real coefficients, starting from rho = I (the identity is
 * propagated instead of I/2^n, Sec. II.C), and applies one elementary gate
 * V_Q = exp(-(theta/2) Q) at a time with the imaginary-time rule of
 * Eq. (ITPP_PropRules): a string anticommuting with Q is unchanged, a
 * commuting string P becomes cosh(theta) P - sinh(theta) Q P.  After every
 * gate the strings are merged, truncated (keep |c| > threshold; above
 * max_terms strings keep the identity and the max_terms-1 largest |c|, ties
 * broken by the smaller canonical key) and divided by the identity
 * coefficient (Algorithm 1; per-gate normalisation as Sec. II.C requires).
 * ITPP_OPT_REAL_TIME switches the gates to the real-time rule of Sec. II.B;
 * itpp_import loads another starting state.
 *
 * Conventions shared by every entry point
 * --------------------------------------
 *  - Pauli strings are packed as W = ceil(n/64) little-endian uint64 words of
 *    x bits followed (in a separate array) by W words of z bits; qubit j is
 *    bit (j % 64) of word (j / 64).  (x,z) = (0,0) I, (1,0) X, (0,1) Z,
 *    (1,1) Y, and P(x,z) = i^{|x & z|} X^x Z^z, so every string is Hermitian.
 *    Arrays of strings are string-major: string s occupies words
 *    [s*W, s*W + W).  Bits at or above n must be zero.
 *  - The canonical key order (used for cap ties and for itpp_export) compares
 *    the x bits as one n-bit integer, then the z bits as one n-bit integer.
 *  - Gate angle: theta = alpha[term] * mult[gate] * dtau, evaluated left to
 *    right in IEEE double; cosh and sinh are taken once per gate on the host.
 *  - All pointers are host pointers, except the arrays of the two *_device
 *    entry points; the caller owns them, the library copies what it needs
 *    during the call and keeps no reference.  Device state is owned by the
 *    context.
 *  - Every call returns an itpp_status; ITPP_OK is 0.  On error nothing is
 *    written to output arguments (except the required capacity that the
 *    export calls report) and itpp_last_error() describes the cause.
 *  - A context is used from one host thread at a time.
 */
#ifndef ITPP_H_
#define ITPP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct itpp_ctx_s* itpp_ctx;

typedef enum {
  ITPP_OK = 0,
  ITPP_ERR_ARG = 1,      /* invalid argument (message says which) */
  ITPP_ERR_OOM = 2,      /* device memory for the requested cap is not available */
  ITPP_ERR_CAP = 3,      /* cap reached under ITPP_CAP_FAIL */
  ITPP_ERR_NUMERIC = 4,  /* identity coefficient not finite or not positive */
  ITPP_ERR_DEVICE = 5,   /* HIP runtime error or missing gfx950 device */
  ITPP_ERR_STATE = 6     /* call out of order (e.g. evolve before set_schedule) */
} itpp_status;

/* Stored coefficient type.  ITPP_F64: binary64 throughout.  ITPP_F32: the
 * coefficients are binary32 and every product and sum of the propagation
 * rule (Eq. ITPP_PropRules) is rounded to binary32 with cosh/sinh rounded to
 * binary32 once per gate; the threshold and cap compare the exactly widened
 * magnitudes; the division by the identity coefficient (Sec. II.C) is done
 * in binary64 and rounded once to binary32; itpp_expect sums in binary64
 * with compensation and itpp_export returns the binary32 values widened. */
typedef enum { ITPP_F64 = 0, ITPP_F32 = 1 } itpp_precision;

/* What to do when more than max_terms strings survive the threshold
 * (Sec. II.C, practical considerations): keep the largest (K-truncation) or
 * stop with ITPP_ERR_CAP. */
typedef enum { ITPP_CAP_TOPK = 0, ITPP_CAP_FAIL = 1 } itpp_cap_policy;

typedef struct {
  int32_t n_qubits;           /* 1..128 */
  int32_t precision;          /* itpp_precision */
  double threshold;           /* delta >= 0, keep |c| > delta (Sec. II.B); delta < 1 */
  int64_t max_terms;          /* K >= 1: the identity plus at most K-1 others */
  int32_t cap_policy;         /* itpp_cap_policy */
  int32_t reserved0;
  void* stream;               /* hipStream_t to run on, or NULL for the null stream */
  int64_t device_bytes_limit; /* 0: no limit; else fail create with ITPP_ERR_OOM above it */
} itpp_config;

typedef struct {
  int64_t n_terms;       /* strings in the current state (after truncation) */
  int64_t n_gates;       /* elementary gates applied by the last evolve */
  double term_updates;   /* sum over those gates of the strings entering the gate */
  double c_identity;     /* identity coefficient before the last normalisation */
  int32_t cap_hit;       /* 1 if the cap truncated at least one gate */
  int32_t reserved0;
  double alg_bytes;      /* sum over gates of (strings in + strings out) * (16W + 8) */
  int64_t spec_gates;    /* gates that wrote only strings above a predicted cap margin */
  int64_t spec_retries;  /* of those, gates redone because the prediction was too high */
  double written;        /* sum over the gates of the strings they stored (identity included;
                            above the cap when speculating: the next gate drops the excess) */
  double c_I_min;        /* smallest and largest identity coefficient before normalisation */
  double c_I_max;        /*   over the gates (Sec. II.C normalisation) */
  double kth_abs_min;    /* smallest K-th largest |c| (normalised) over the gates whose cap
                            bound (K-truncation, Sec. II.C); +inf if none */
  int64_t graph_steps;   /* Trotter steps of this call launched as replays of a
                            recorded step graph (ITPP_OPT_GRAPHS); a replay cut short
                            by a redone speculative gate counts too, so with redos
                            this can exceed the steps of the call */
} itpp_stats;

/* Kernel timing gathered with HIP events on the context's stream while
 * enabled (itpp_set_timing): total milliseconds and launch counts of the
 * gate kernel and of the truncation-selection kernels, and the algorithmic
 * bytes of the timed gates (strings in + strings out times 16W + 8). */
typedef struct {
  double gate_ms;
  double select_ms;
  int64_t gate_launches;
  double alg_bytes;
} itpp_timing;

/* Create a context on the current HIP device.  Validation (ITPP_ERR_ARG):
 * n_qubits outside 1..128, threshold negative, not finite or >= 1,
 * max_terms < 1, unknown precision or cap policy.  ITPP_ERR_DEVICE if no
 * gfx950 device is current.  Allocates the state buffers (about
 * 8 * max_terms * (16W + 8) bytes); ITPP_ERR_OOM if that fails or exceeds
 * device_bytes_limit.  The state starts as rho = I. */
itpp_status itpp_create(const itpp_config* cfg, itpp_ctx* out);

/* Free the context and its device memory.  NULL is accepted. */
itpp_status itpp_destroy(itpp_ctx ctx);

/* Hamiltonian H = sum_k alpha_k Q_k (Algorithm 1 input).  x, z: n_terms*W
 * words each; alpha: n_terms finite doubles.  A term may flip at most two
 * bits (|x| + |z| <= 2 over its words: one- and two-letter X/Z terms and
 * single-site Y); others give ITPP_ERR_ARG.  Identity terms are accepted and
 * skipped as gates.  Replaces any previous Hamiltonian and schedule. */
itpp_status itpp_set_hamiltonian(itpp_ctx ctx, int32_t n_terms, const uint64_t* x,
                                 const uint64_t* z, const double* alpha);

/* One Trotter step as a gate list: gate g applies term term_idx[g] with
 * multiplier mult[g] (first order: every term once with 1; Strang: A at 1/2,
 * B at 1, A at 1/2; Sec. II.C).  Indices must be in range, mult finite. */
itpp_status itpp_set_schedule(itpp_ctx ctx, int32_t n_gates, const int32_t* term_idx,
                              const double* mult);

/* Reset the state to rho = I (a single identity string with coefficient 1). */
itpp_status itpp_reset(itpp_ctx ctx);

/* Replace the state by rho proportional to sum_j coef[j] P_j (the Pauli-basis
 * expansion of Sec. II.B, Eq. Observable_Pauli) and restart the schedule at
 * its first gate.
 * x, z: n_strings * W canonical words each, in the layout itpp_export writes;
 * coef: n_strings values.  Host arrays, copied during the call.
 * - The identity must be present with a coefficient above max(0, threshold).
 *   The state is normalised by it (Sec. II.C): itpp_export then returns
 *   coef[j] / coef[identity].
 * - Other strings with |coef| at or below the threshold are dropped (every
 *   stored value exceeds it, Sec. II.B).  At most max_terms strings may remain.
 * - Strings must be distinct, with no bits at or above n_qubits; coefficients
 *   must be finite.  An ITPP_F32 context rounds them to binary32 first (the
 *   threshold and identity tests then apply to the rounded values).
 * - Needs a schedule: the stored layout depends on its first two gates.  A
 *   later itpp_set_hamiltonian or itpp_set_schedule returns to rho = I.
 * ITPP_ERR_ARG on bad input (the previous state is kept), ITPP_ERR_STATE
 * without a schedule, ITPP_ERR_DEVICE on a HIP error (then no valid state
 * remains until itpp_reset). */
itpp_status itpp_import(itpp_ctx ctx, int64_t n_strings, const uint64_t* x, const uint64_t* z,
                        const double* coef);

/* Apply n_steps Trotter steps of the schedule with step dtau > 0 (finite).
 * Runs asynchronously on cfg.stream except for the final status check; st
 * (nullable) receives the statistics of this call.  ITPP_ERR_CAP under
 * ITPP_CAP_FAIL when a gate leaves more than max_terms strings;
 * ITPP_ERR_NUMERIC if the identity coefficient is not finite and positive.
 * After either error the state is invalid until itpp_reset. */
itpp_status itpp_evolve(itpp_ctx ctx, double dtau, int64_t n_steps, itpp_stats* st);

/* Apply the next n_gates elementary gates of the schedule (continuing
 * inside a Trotter step if the previous call stopped there); same semantics
 * and errors as itpp_evolve, which applies n_steps times the schedule's
 * non-identity gates.  Lets a caller inspect or checkpoint the state after
 * any elementary gate of Algorithm 1. */
itpp_status itpp_evolve_gates(itpp_ctx ctx, double dtau, int64_t n_gates, itpp_stats* st);

/* <O> = sum_j coef[j] * a_{P_j} for O = sum_j coef[j] P_j (Eq.
 * Expectation_Value in the Pauli basis; absent strings count 0), summed in
 * FP64 with compensation on the device.  out receives one double. */
itpp_status itpp_expect(itpp_ctx ctx, int32_t n_strings, const uint64_t* x, const uint64_t* z,
                        const double* coef, double* out);

/* Number of strings in the current (truncated) state, identity included. */
itpp_status itpp_num_terms(itpp_ctx ctx, int64_t* out);

/* Copy the current state in ascending canonical key order: x, z receive
 * n*W words each, coef n normalised coefficients (identity = 1).  If
 * capacity is smaller than the number of strings, nothing is copied and
 * *n_out receives the required capacity with ITPP_ERR_ARG. */
itpp_status itpp_export(itpp_ctx ctx, int64_t capacity, uint64_t* x, uint64_t* z, double* coef,
                        int64_t* n_out);

/* Squared-state estimate of Sec. II.C: <O>_{2 tau} ~= Tr[(O rho) rho] /
 * Tr[rho^2] for the current state rho (imaginary time tau), without forming
 * rho^2.  With rho = 2^-n sum_P a_P P (a_I = 1) and O = sum_j coef[j] Q_j:
 * *purity = sum_P a_P^2 (= 2^n Tr[rho^2], the l2 norm of the coefficients)
 * and *value = (sum_j coef[j] sum_P a_P a_R s) / *purity, where Q_j P = s R
 * for the strings P that commute with Q_j (s = +-1; the others cancel in
 * pairs).  Strings in the same layout as itpp_expect; any weight.  Host
 * arrays; waits for the stream.  Cost grows with n_strings times the number
 * of stored strings (one binary search per commuting pair). */
itpp_status itpp_expect_squared(itpp_ctx ctx, int32_t n_strings, const uint64_t* x, const uint64_t* z,
                                const double* coef, double* value, double* purity);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as itpp_expect_squared, bit for bit, computed without any device or
 * host allocation.  The observable words are staged, their tables built and
 * the per-block partial sums kept in a fixed scratch area of the library
 * (about 1.4 MiB per GPU, held until the process ends) instead of buffers
 * allocated per call.  Limits: n_strings <= 4096 and at most 65536
 * non-identity sites summed over the strings (ITPP_ERR_ARG beyond either).
 * Every call on one GPU uses that GPU's single scratch area: calls that
 * overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller.  Host arrays; waits for the stream. */
itpp_status itpp_expect_squared_noalloc(itpp_ctx ctx, int32_t n_strings, const uint64_t* x, const uint64_t* z,
                                       const double* coef, double* value, double* purity);

/* Device-pointer variants, for arrays that already live on the device (for
 * example torch tensors).  Both run on cfg.stream; the arrays must be ready
 * on that stream and stay valid until the work is done.
 *
 * itpp_expect_device: as itpp_expect with x, z, coef and out in device
 * memory.  Enqueued without waiting: out holds <O> once cfg.stream reaches
 * this point.  Bits at or above n_qubits cannot be checked and are ignored.
 *
 * itpp_export_device: the surviving strings (canonical words, normalised
 * coefficients as itpp_export) written to device arrays of at least
 * capacity strings, in storage order (unspecified; itpp_export sorts them).
 * Waits for the stream; n_out (host) receives the count, also when the
 * capacity is too small (then ITPP_ERR_ARG and nothing is written). */
itpp_status itpp_expect_device(itpp_ctx ctx, int32_t n_strings, const uint64_t* x, const uint64_t* z,
                               const double* coef, double* out);
itpp_status itpp_export_device(itpp_ctx ctx, int64_t capacity, uint64_t* x, uint64_t* z, double* coef,
                               int64_t* n_out);

/* Reverse sweep (derivatives of an observable with the truncation support
 * held fixed).  The forward map of Algorithm 1 is differentiated gate by
 * gate: for the division by the identity coefficient b_I,
 * dL/db_P = lambda'_P / b_I minus, at the identity only, sum_R lambda'_R a'_R
 * / b_I; the kept set restricts that vector; the gate rule of Eq.
 * ITPP_PropRules gives lambda_P = ch lambda_u[P] - sigma sh lambda_u[R] for a
 * commuting P (Q P = sigma R) and lambda_P = lambda_u[P] otherwise, and
 * dL/dtheta = sum over commuting P of a_P (sh lambda_u[P] - sigma ch
 * lambda_u[R]).  With theta = alpha_k m dtau the chain rule gives dL/dalpha_k
 * and dL/ddtau.
 *
 * itpp_set_adjoint: every_steps > 0 makes the following forward runs store a
 * packed copy of the state every every_steps Trotter steps (and run without
 * speculation, so recomputation reproduces every stored layout);
 * workspace_bytes bounds the device memory of one itpp_backward call for its
 * recomputed states (0: 70% of the free device memory).  ITPP_F64 contexts
 * only (ITPP_ERR_ARG otherwise).  Takes effect for the gates applied after
 * the next reset, set_schedule or itpp_import. */
itpp_status itpp_set_adjoint(itpp_ctx ctx, int32_t every_steps, int64_t workspace_bytes);

/* For L = sum_j coef[j] a_{P_j} of the current state (strings as in
 * itpp_expect): *value = L, d_alpha[k] = dL/dalpha_k for every Hamiltonian
 * term (n_terms doubles, zero for identity terms and unscheduled terms),
 * *d_dtau = dL/ddtau, and, if d_theta is not NULL, dL/dtheta for every
 * elementary gate applied since the last reset or itpp_import (in order):
 * d_theta_capacity doubles are available there, and ITPP_ERR_ARG is returned
 * (nothing written) when that is fewer than the gates (itpp_num_gates).
 * Requires a forward run since then with itpp_set_adjoint enabled, one dtau
 * and imaginary-time gates only (ITPP_ERR_STATE otherwise).  Between the stored copies the states are
 * recomputed: once, when every state of a segment fits in the workspace
 * (each at most 2 * max_terms + 1 strings), else twice, with sub-checkpoints
 * every ~sqrt(segment) gates; ITPP_ERR_OOM if the workspace cannot hold
 * those.  The current state is the same after the
 * call; after an error it needs a reset. */
itpp_status itpp_backward(itpp_ctx ctx, int32_t n_strings, const uint64_t* x, const uint64_t* z,
                          const double* coef, double* value, double* d_alpha, double* d_dtau, double* d_theta,
                          int64_t d_theta_capacity);

/* Elementary gates applied since the last reset, itpp_set_schedule or
 * itpp_import (the length of itpp_backward's d_theta). */
itpp_status itpp_num_gates(itpp_ctx ctx, int64_t* out);

/* Engine options (results do not depend on them; only speed does).
 *  ITPP_OPT_SPECULATION (default 1): once the cap binds, a gate writes only
 *    the strings above a margin below the K-th value predicted from the
 *    previous gate; if fewer than K-1 strings pass, the gate is redone
 *    without the margin, so the kept set is always the exact one.
 *  ITPP_OPT_SPEC_MARGIN (default 0.98): that margin as a factor in (0, 1].
 *  ITPP_OPT_GATE_SHAPE (default 3): the gate kernel's launch shape.
 *    0 = one 1024-thread workgroup per CU with 4000 (n <= 64) or 2000
 *    (n <= 128) strings per tile; 1 = two 512-thread workgroups per CU with
 *    2380 or 1500 strings per tile; 2 = the 256-thread layer kernel with
 *    1022 strings per tile (runs as 1 while a weight cutoff is set); 3 =
 *    automatic: 2 while the stored state held at most 2^19 strings at the
 *    host's last synchronisation (every 512 gates), 1 above, and 1 with
 *    forward checkpoints (itpp_set_adjoint).  Measured on one MI355X, 2 is
 *    ahead up to 2^18 strings and 1 from 2^20 on.
 * One option changes the method instead:
 *  ITPP_OPT_REAL_TIME (default 0): 1 applies the real-time rule of Sec. II.B
 *    to the following gates, U_Q(theta)^dagger P U_Q(theta) with
 *    U_Q = exp(-i theta Q / 2) and theta = alpha_k * mult * dtau: commuting
 *    strings pass unchanged, anticommuting ones become
 *    cos(theta) P + i sin(theta) Q P (real: i Q P = -+R).  Truncation is
 *    unchanged; the identity coefficient stays 1.  Start from a state given
 *    by itpp_import (rho = I does not move).  Disables the reverse sweep of
 *    the run.
 *  ITPP_OPT_GRAPHS (default 1): run whole Trotter steps as replays of a HIP
 *    graph recorded from the context's own launches.  From the second step
 *    on every step starts from the same bit order of the stored keys, so
 *    its launches are the same; the library records them once (stream
 *    capture) and replays them (two steps per graph where a step has an
 *    odd number of non-identity gates).  Used only with speculation on, no
 *    forward checkpoints (itpp_set_adjoint) and no event timing
 *    (itpp_set_timing).
 *    The null stream cannot be captured: with cfg.stream == NULL the gates
 *    of an itpp_evolve run on a private non-blocking stream that waits for
 *    the null stream's earlier work and that the null stream then waits
 *    for, so the ordering seen by the caller is unchanged.  Results are
 *    bit-identical with and without graphs.  Changing an option, the
 *    Hamiltonian or the schedule drops the recorded graph.
 *  ITPP_OPT_GRID_DIV (default 1; 1, 2, 4 or 8): the gate kernel launches the
 *    workgroups that fit on the device at once divided by this (its tiles
 *    are taken from a ticket counter, so any grid covers every tile).
 *    Smaller grids leave room for the kernels of other contexts running
 *    concurrently (the batch); results do not depend on it.
 *  ITPP_OPT_MAX_WEIGHT (default 0 = none; an integer in [0, n]): the Pauli
 *    weight cutoff of Sec. II.B.  From the next gate on, an output string
 *    with more non-identity letters than the cutoff is dropped, with the
 *    coefficient threshold and before the cap selection (the K kept strings
 *    are the largest within the cutoff; the identity always passes).  The
 *    strings of the current state are not filtered until a gate produces
 *    them.  Gates of shape 2 run on shape 1 while a cutoff is set.  Not
 *    available with the reverse sweep (ITPP_ERR_STATE with checkpoints
 *    set, and itpp_set_adjoint refuses while a cutoff is set). */
typedef enum {
  ITPP_OPT_SPECULATION = 1,
  ITPP_OPT_SPEC_MARGIN = 2,
  ITPP_OPT_GATE_SHAPE = 3,
  ITPP_OPT_REAL_TIME = 4,
  ITPP_OPT_GRAPHS = 5,
  ITPP_OPT_GRID_DIV = 6,
  ITPP_OPT_MAX_WEIGHT = 7
} itpp_option;
itpp_status itpp_set_option(itpp_ctx ctx, int32_t option, double value);

/* Enable (1) or disable (0) per-gate HIP event timing; enabling clears the
 * accumulated figures.  Timing adds two event records per gate. */
itpp_status itpp_set_timing(itpp_ctx ctx, int32_t enable);

/* Wait for the stream and return the accumulated timing. */
itpp_status itpp_get_timing(itpp_ctx ctx, itpp_timing* out);

/* Batches of independent instances (the same method on many Hamiltonians,
 * steps and sizes at once).  itpp_batch_create makes n_inst contexts from
 * cfgs[i] (each cfg as for itpp_create; its stream field is ignored: every
 * instance gets a stream of its own) whose device buffers are consecutive
 * slices of one allocation sized to the sum of their needs.  The instances
 * are ordinary contexts: itpp_batch_instance returns instance i (owned by
 * the batch; do not destroy it) for set_hamiltonian, set_schedule,
 * set_option, expect, export, ...  Every instance computes exactly what a
 * single context with the same configuration computes.
 * ITPP_ERR_ARG for n_inst < 1 or a bad configuration, ITPP_ERR_OOM if the
 * arena cannot be allocated. */
typedef struct itpp_batch_s* itpp_batch;
itpp_status itpp_batch_create(int32_t n_inst, const itpp_config* cfgs, itpp_batch* out);
itpp_status itpp_batch_destroy(itpp_batch b);
itpp_ctx itpp_batch_instance(itpp_batch b, int32_t i);

/* Host worker threads that drive the instances' streams (1..64, default 4). */
itpp_status itpp_batch_set_workers(itpp_batch b, int32_t workers);

/* Evolve instance i by n_steps[i] Trotter steps of dtau[i] (as itpp_evolve),
 * all instances concurrently; st (NULL or n_inst entries) receives each
 * instance's statistics.  Returns the first instance error (message from
 * itpp_batch_last_error). */
itpp_status itpp_batch_evolve(itpp_batch b, const double* dtau, const int64_t* n_steps, itpp_stats* st);

/* Autotuner, by coordinate descent: first the gate kernel shape
 * (ITPP_OPT_GATE_SHAPE 0, 1 or 2, chosen separately for instances with
 * n <= 64 and n > 64; nine pairs), then the worker count (2, 4, 8, 16),
 * then the grid divisor (ITPP_OPT_GRID_DIV 1, 2, 4, 8).  Each probe resets
 * all instances, applies warm_gates gates untimed, then times probe_gates
 * more gates on every instance and scores term updates per second.  The
 * best setting is written to the non-NULL outputs (best_shape = shape for
 * n <= 64 + 3 * shape for n > 64) and left applied, every instance reset. */
itpp_status itpp_batch_autotune(itpp_batch b, const double* dtau, int64_t warm_gates, int64_t probe_gates,
                                int32_t* best_shape, int32_t* best_workers, int32_t* best_grid_div,
                                double* best_rate);

/* Message for the last batch error (b == NULL: last creation failure). */
const char* itpp_batch_last_error(itpp_batch b);

/* Message for the last error on ctx (for ctx == NULL: the last itpp_create
 * failure of this thread). */
const char* itpp_last_error(itpp_ctx ctx);

/* Library build information ("gfx950 ..."). */
const char* itpp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ITPP_H_ */
