/*
 * nisqtol.h -- C ABI of libnisqtol: Monte Carlo state-vector simulation of a
 * quantum circuit under the Pauli error model on an AMD Instinct MI355X
 * (gfx950), following ArsoNISQ (Brandhofer, Devitt, Polian; arXiv 2301.07264).
 *
 * The paper's framework takes a circuit, a success criterion and either a
 * Pauli error rate (-> success probability) or a target success probability
 * (-> tolerable error rate) (Sec. IV).  Its Monte Carlo branch simulates the
 * circuit N times; after every one-qubit gate an X, Z or Y error happens with
 * probabilities p_X, p_Z, p_Y, and after a two-qubit gate the same happens
 * independently on each of its qubits (Sec. IV-B.2).  An error is an error
 * gate appended after the gate (Sec. IV-B); Eq. 2 gives the single-qubit
 * actions.  Success probability is the mean of the criterion over the
 * simulated states (Sec. IV-C); the tolerable rate is where it meets the
 * target (Sec. IV-D, Fig. 3).
 *
 * Conventions
 *   - Amplitude k of an n-qubit state belongs to basis state |k>; qubit 0 is
 *     the least-significant bit of k.  Amplitudes are interleaved complex:
 *     NT_C64 = 2 x float per amplitude, NT_C128 = 2 x double.
 *   - Error sites: one per qubit a gate touches, numbered in gate order and,
 *     within a gate, in the order its qubits are listed (the k + 2m error
 *     locations of Sec. IV-B.1).  "Error rate" p is per site; the uniform
 *     model is p_X = p_Y = p_Z = p/3 (Sec. IV-D, Sec. V).
 *   - Random draws: Philox4x64-10 (Salmon et al., SC'11), key = (seed,
 *     circuit id), counter = (site, trajectory, 0, 0).  A site fires iff
 *     word0 < floor((p_x+p_y+p_z) * 2^64) (always when the sum is >= 1); its
 *     Pauli is X if word1 < c_X, else Y if word1 < c_XY, else Z.  When
 *     p_x == p_y == p_z (the uniform model of every sweep and search),
 *     c_X = floor(2^64 / 3) and c_XY = floor(2^64 * 2/3), the thresholds of
 *     the correctly rounded doubles 1/3 and 2/3, at every rate; otherwise
 *     c_X = floor(p_x/sum * 2^64) and c_XY = floor((p_x+p_y)/sum * 2^64),
 *     each fraction rounded once in IEEE FP64 (a fraction >= 1 means
 *     "always").  Rates are not part of the counter, so the fired sets of one
 *     trajectory are nested across rates, with the same Pauli types.
 *   - Fidelity criterion: F = |<R|psi>|^2 / (<R|R><psi|psi>) against the
 *     error-free final state R of the same precision; a trajectory succeeds
 *     iff F >= tau (Sec. II criteria; Sec. IV-C).
 *   - The errors a trajectory sees are a pure function of (circuit, error
 *     model, seed, trajectory index): batching, tiling, fusion and the pass
 *     plan never change them.  Values are a function of those and the plan
 *     (tile width, fusion width; nt_circuit_set_tile / _set_fusion /
 *     nt_autotune_plan), which changes them at rounding level only; with a
 *     fixed plan they are reproducible bit for bit, and batching never
 *     changes them.
 *
 * Errors: every call returns an nt_status; no C++ exception crosses the ABI.
 * nt_last_error() returns a thread-local message for the last failure.
 * Threading: one host thread at a time per context.  Host outputs are
 * complete when a call returns; device outputs are ordered on the context's
 * stream.
 */
#ifndef NISQTOL_H
#define NISQTOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nt_status {
  NT_OK = 0,
  NT_ERR_INVALID_ARG = 1,      /* bad argument; nothing was changed */
  NT_ERR_UNSUPPORTED = 2,      /* valid request the library cannot serve */
  NT_ERR_OUT_OF_MEMORY = 3,    /* size check failed before any allocation, or an allocation failed */
  NT_ERR_DEVICE = 4,           /* HIP runtime error; message carries hipGetErrorString */
  NT_ERR_BUFFER_TOO_SMALL = 5, /* required size returned through the size argument */
  NT_ERR_NOT_BRACKETED = 6     /* tolerable-rate search: target not inside [p_lo, p_hi] */
} nt_status;

/* Amplitude precision (nt_set_precision). */
enum { NT_C64 = 1, NT_C128 = 2 };

/* Gate kinds.  R_P(theta) = exp(-i theta P/2); U(a,b,c) = Rz(a) Ry(b) Rz(c)
 * as one gate with one error site; CNOT lists (control, target); CP(phi)
 * multiplies the |11> component by e^{i phi}; RZZ(g) = exp(-i g Z(x)Z/2);
 * U1Q/U2Q take a caller matrix, row-major complex (re, im interleaved), the
 * 4x4 one on local index b_q0 + 2*b_q1. */
enum nt_gate_kind {
  NT_H = 0, NT_X = 1, NT_Y = 2, NT_Z = 3, NT_S = 4, NT_T = 5,
  NT_RX = 6, NT_RY = 7, NT_RZ = 8, NT_U = 9, NT_U1Q = 10,
  NT_CNOT = 11, NT_CZ = 12, NT_CP = 13, NT_SWAP = 14, NT_RZZ = 15, NT_U2Q = 16,
  NT_NUM_GATE_KINDS = 17
};

typedef struct nt_gate {
  uint16_t kind;          /* enum nt_gate_kind */
  uint8_t nq;             /* 1 or 2; must match the kind */
  uint8_t pad;
  int32_t q[2];           /* qubits; q[1] unused for one-qubit kinds */
  double param[3];        /* angles (radians) as the kind requires */
  const double *matrix;   /* U1Q: 8 doubles, U2Q: 32 doubles; else NULL */
} nt_gate;

typedef struct nt_ctx nt_ctx;
typedef struct nt_circuit nt_circuit;

/* ---- context ------------------------------------------------------------ */

/* Opens HIP device `device`.  hip_stream: a hipStream_t to launch on (for
 * example torch.cuda.current_stream().cuda_stream), or NULL to let the
 * library create and own a default-priority stream.  Fails with
 * NT_ERR_DEVICE when no device is present. */
nt_status nt_create(nt_ctx **out, int device, void *hip_stream);

/* Frees every library-owned device buffer and the owned stream. */
void nt_destroy(nt_ctx *ctx);

/* Error model (Sec. IV-B.2): after every gate, on each touched qubit, X with
 * p_x, Y with p_y, Z with p_z.  Needs each >= 0 and p_x+p_y+p_z <= 1.
 * Default: all zero. */
nt_status nt_set_error_model(nt_ctx *ctx, double p_x, double p_y, double p_z);

/* NT_C64 (float amplitudes; FP64 overlaps, norms and counts) or NT_C128.
 * Default NT_C128. */
nt_status nt_set_precision(nt_ctx *ctx, int prec);

/* Upper bound on trajectories simulated concurrently (each holds one state
 * vector in device memory).  0 = automatic (memory-bounded).  Does not change
 * results. */
nt_status nt_set_max_batch(nt_ctx *ctx, uint64_t max_batch);

/* ---- circuits (host objects; ctx may be NULL) ---------------------------- */

/* Copies gates[0..n_gates) after validating qubits (0 <= q < n, distinct for
 * two-qubit kinds), kinds, arity and matrices.  1 <= n_qubits <= 32.
 * 0 <= n_gates <= 2^19 (NT_ERR_UNSUPPORTED above: the device event words
 * hold an op index in 20 bits, and a plan may add one no-op per gate). */
nt_status nt_circuit_load(nt_ctx *ctx, int n_qubits, const nt_gate *gates, int64_t n_gates,
                          nt_circuit **out);

/* Text format: "qubits <n>" then one gate per line, "NAME q0 [q1] [angles]",
 * U1Q/U2Q followed by the row-major (re im) matrix entries; '#' comments. */
nt_status nt_circuit_load_text(nt_ctx *ctx, const char *path, nt_circuit **out);

void nt_circuit_free(nt_circuit *c);

/* n qubits, G gates, S error sites (k + 2m, Sec. IV-B.1). */
nt_status nt_circuit_info(const nt_circuit *c, int *n, int64_t *G, int64_t *S);

/* Second Philox key word (default 0), so that many circuits under one seed
 * draw independent errors. */
nt_status nt_circuit_set_id(nt_circuit *c, uint64_t circuit_id);

/* Tile width (qubits per work-group tile) of the circuit's plan at precision
 * `prec`: 0 = automatic (a fixed cost model of the pass count; complex64
 * takes 2^12-amplitude tiles when their predicted pass cost is at least 5%
 * lower than 2^13), else a width in [min(n, 10), min(n, 13)] (complex64) or
 * [min(n, 10), min(n, 12)] (complex128).  The tile width changes which
 * commuting gates a pass groups, so results change at rounding level only;
 * with a fixed width they are reproducible.  NT_ERR_INVALID_ARG outside the
 * range. */
nt_status nt_circuit_set_tile(nt_circuit *c, int prec, int tile_qubits);

/* Gate fusion of the circuit's plan at precision `prec`: 0 = automatic
 * (currently 2), 1 = none (one op per gate), 2 = two-qubit blocks and
 * diagonal runs, 3 = two-qubit blocks only, 4 = diagonal runs only; at
 * complex64 the widths with blocks also join four RX-type one-qubit gates,
 * one on each register qubit, into one op.  Within
 * a pass, a two-qubit gate takes the runs of
 * one-qubit gates right before it on its qubits (not already taken) and,
 * when it took any, the runs right after it, and the block is applied as one
 * dense 4x4 (both qubits then sit in registers) when a cost model prices it
 * below its gates; a dense two-qubit gate (U2Q) forms such a block even
 * alone (at every width a SWAP is a permutation of two register qubits).  Within a register segment, runs of at least three
 * diagonal gates (each with at most one qubit in the registers) multiply
 * every amplitude once by the product of their phases.  An error inside a
 * block or run still acts right after its gate (Sec. IV-B): a trajectory
 * with such an error applies that block gate by gate, and a run takes each
 * gate's phase under the errors before it.  Results change at rounding
 * level only.  NT_ERR_INVALID_ARG for other widths. */
nt_status nt_circuit_set_fusion(nt_circuit *c, int prec, int width);

/* Autotuner: runs n_traj trajectories (seed, current error model) with each
 * allowed tile width from the largest down to two below it, keeps the
 * fastest as the circuit's tile width (nt_circuit_set_tile) and returns it.
 * ms_out (may be NULL): milliseconds per candidate, in the order tried
 * (up to 3 entries). */
nt_status nt_autotune(nt_ctx *ctx, nt_circuit *c, uint64_t seed, uint64_t n_traj, int *tile_out,
                      double *ms_out);

/* Autotuner over the plan: tile width and gate fusion together.  Runs n_traj
 * trajectories (seed, current error model and precision) for each tile
 * width from the largest down to two below it and each fusion width in
 * {2, 3, 4, 1} (nt_circuit_set_fusion), keeps the fastest pair as the
 * circuit's tile width and fusion width at the context's precision and
 * returns it.  ms_out (may be NULL): milliseconds per candidate, tile-major in
 * the order tried, at most ms_cap entries written.  Values are those of the
 * chosen plan (plans differ at rounding level only). */
nt_status nt_autotune_plan(nt_ctx *ctx, nt_circuit *c, uint64_t seed, uint64_t n_traj, int *tile_out,
                           int *fusion_out, double *ms_out, int ms_cap);

/* Host-only view of the gate-pass plan used for precision `prec`: number of
 * HBM passes over a state vector per trajectory, LDS segments, and the
 * local-tile width in qubits. */
nt_status nt_plan_info(const nt_circuit *c, int prec, int *n_passes, int *n_segments,
                       int *tile_qubits);

/* Host-only export of that plan, for checking it: for each gate in
 * application order its gate index, pass and segment (arrays of n_gates; the
 * gates of a fused block appear in the order the block applies them); the
 * local-qubit mask of each pass (n_passes) and the register-qubit mask of
 * each segment (n_segments).  Any pointer may be NULL; sizes must match
 * nt_plan_info. */
nt_status nt_plan_export(const nt_circuit *c, int prec, int32_t *op_gate, int32_t *op_pass,
                         int32_t *op_segment, uint64_t *pass_local_mask, uint64_t *segment_reg_mask);

/* Host-only: ops the plan runs per trajectory (a fused op counts once;
 * no-op pads that keep fused ops at even positions of their segments
 * included) and the number of fused ops (two-qubit blocks, diagonal runs
 * and one-qubit layers). */
nt_status nt_plan_ops(const nt_circuit *c, int prec, int64_t *n_ops, int64_t *n_fused);

/* ---- success criterion (Sec. II, Sec. V) ----------------------------------- */

/* Criterion every scoring call of the context evaluates on a final state psi
 * (R = the error-free state):
 * NT_CRIT_FIDELITY    -- F = |<R|psi>|^2 / (<R|R><psi|psi>); a state succeeds
 *                        when F >= tau.  Default.
 * NT_CRIT_TARGET_PROB -- probability of measuring basis state `target`,
 *                        |psi_target|^2 / <psi|psi> (circuits with a single
 *                        correct outcome).
 * NT_CRIT_HEAVY       -- heavy-output probability: the mass of psi on the
 *                        basis states whose error-free probability |R_k|^2
 *                        exceeds the median of all 2^n of them (the mean of
 *                        the two middle values); quantum-volume binning.
 * For the two probability criteria a state's success is that probability
 * itself: success probabilities are means over trajectories (and per error
 * type in the exhaustive branch), while count_out still counts values >= tau.
 * The heavy set is decided on the device's reference state in FP64; the
 * median is selected exactly, once per circuit and precision.
 * `target` is checked against the circuit at run time (NT_ERR_INVALID_ARG).
 * The last-error short-cut does not apply to these two criteria (they are
 * not invariant under the error-free rest of the circuit) and is skipped. */
enum { NT_CRIT_FIDELITY = 0, NT_CRIT_TARGET_PROB = 1, NT_CRIT_HEAVY = 2 };
nt_status nt_set_criterion(nt_ctx *ctx, int criterion, uint64_t target);

/* ---- Monte Carlo runs ------------------------------------------------------ */

/* Runs trajectories [traj_begin, traj_begin + n_traj) under the current
 * error model and precision and scores each against the error-free state
 * (Sec. IV-B.2, IV-C) by the context's criterion.  fid_out: n_traj doubles
 * (the criterion value of each trajectory), host or device memory, may be
 * NULL.  count_out: number of trajectories with value >= tau (may be NULL).
 * p_out (may be NULL): success probability, count / n_traj for the fidelity
 * criterion, the mean value for the probability criteria. */
nt_status nt_run(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t traj_begin,
                 uint64_t n_traj, double tau, double *fid_out, uint64_t *count_out,
                 double *p_out);

/* nt_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same trajectories, scoring and outputs as nt_run with the short-cuts off
 * (short-cut flags are ignored here), but no hipMalloc, hipFree or other
 * allocating routine is called.  Every device buffer of the call (the
 * circuit's plan tables and error-free reference state, rebuilt on every
 * call, and the per-trajectory events, states, partials and frames) lives in
 * one static scratch array of 64 MiB per device, held until the process
 * ends.  Limit: the plan tables, the reference state and one trajectory's
 * buffers must fit in it (complex64 states up to about 2^21 amplitudes);
 * larger requests fail with NT_ERR_UNSUPPORTED before any launch.
 * Trajectories run in chunks that fit.  All calls on one device share its
 * array and the last call's contents stay in it: calls that overlap on one
 * device (several contexts or threads) race.  Arguments and outputs as in
 * nt_run. */
nt_status nt_run_noalloc(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t traj_begin,
                         uint64_t n_traj, double tau, double *fid_out, uint64_t *count_out,
                         double *p_out);

/* Batched Monte Carlo over many independent circuits (instances of
 * different sizes): for each circuit i, trajectories [traj_begin,
 * traj_begin + n_traj) under the context's error model, precision and
 * criterion, with Philox key (seed, circuit id of circuits[i]).  Values are
 * bit-identical to nt_run on each circuit alone under the same settings
 * (short-cuts included: zero-fired trajectories of the shared launches are
 * not simulated under the fidelity criterion; larger circuits take the
 * short-cut path of nt_run).
 * Circuits whose plan is a single pass over one tile share launches (one
 * work-group per trajectory, per-circuit plan tables); larger ones run back
 * to back without host synchronization.
 * circuits: n_circ handles (a handle may repeat).  vals_out: [n_circ][n_traj]
 * doubles, host or device, may be NULL.  count_out, p_out: n_circ entries on
 * the host, may be NULL; p_out as in nt_run.  Device memory: the reference
 * states of the circuits (held in the context's plan cache) plus one batch
 * of trajectory states for the largest circuit. */
nt_status nt_run_batch(nt_ctx *ctx, const nt_circuit *const *circuits, int n_circ, uint64_t seed,
                       uint64_t traj_begin, uint64_t n_traj, double tau, double *vals_out,
                       uint64_t *count_out, double *p_out);

/* Success probability at each uniform rate rates[r] (p/3 per Pauli) with the
 * same trajectories [0, n_traj) at every rate.  p_out: R doubles (host).
 * The context's error model is left unchanged. */
nt_status nt_sweep(nt_ctx *ctx, const nt_circuit *c, const double *rates, int R, uint64_t seed,
                   uint64_t n_traj, double tau, double *p_out);

/* The plain sweep route to the tolerable rate: nt_sweep at the ascending
 * rates[0..R), then the rate where the success curve, linear in log10 p
 * between grid points, first falls below P_target (rates[0] if it starts
 * below, rates[R-1] if it never does).  p_out: R doubles (host, may be
 * NULL). */
nt_status nt_sweep_crossing(nt_ctx *ctx, const nt_circuit *c, const double *rates, int R, uint64_t seed,
                            uint64_t n_traj, double tau, double P_target, double *p_out, double *p_star);

/* Tolerable uniform rate (Sec. IV-D, Monte Carlo branch, Fig. 3).  The paper
 * names Powell's method without its settings; here: a safeguarded regula
 * falsi (Illinois) in x = log10(p) on f = P(10^x) - P_target over the
 * bracket [p_lo, p_hi], with the same trajectories [0, n_traj) at every
 * probe.  Each step probes the secant root of the bracket (its midpoint if
 * the root falls outside); an end kept twice in a row has its f halved.
 * Returns the first probe whose success probability is within tol of
 * P_target, else the bracket midpoint once p_hi/p_lo <= 1.001.
 * NT_ERR_NOT_BRACKETED if P(p_lo) < P_target or P(p_hi) > P_target.
 * *n_probes counts every Monte Carlo evaluation, including the two ends. */
nt_status nt_tolerable_rate(nt_ctx *ctx, const nt_circuit *c, double P_target, double tol,
                            double p_lo, double p_hi, uint64_t seed, uint64_t n_traj,
                            double tau, double *p_star, int *n_probes);

/* Tolerable uniform rate without a caller's bracket: the search of
 * nt_tolerable_rate (Sec. IV-D) in two stages over the same trajectories.
 *  1. Coarse: nt_tolerable_rate on the first max(1, n_traj/5) trajectories,
 *     in [p0/2, min(2 p0, 1/G)], then [p0/2, 1/G], [1e-6, 1/G], [1e-6, 0.5]
 *     until one holds the target.  p0 = 1 - P_target^(1/S): a trajectory with
 *     no fired site succeeds under the fidelity criterion, so
 *     P(p) >= (1 - p)^S and the tolerable rate is at least p0; 1/G is the
 *     paper's bound (Sec. IV-D); at 2 p0, P would be P_target^2 if every
 *     error were fatal.
 *  2. Full: one probe with all n_traj trajectories at the coarse answer p_c,
 *     the answer if within tol of P_target; else one Newton step in log10 p
 *     with the slope of the coarse bracket, the answer if within tol; else
 *     nt_tolerable_rate between the two probes (or a tenth of a decade from
 *     p_c on the side its probe points to), falling back to the stage-1
 *     brackets, all with n_traj trajectories.
 * The answer always has a full-sample success probability within tol of
 * P_target (or is the midpoint of a bracket narrower than 0.1%).  Cheap with
 * NT_SHORTCUT_REUSE on: the coarse trajectories and rates probed again are
 * not simulated again.  *n_coarse / *n_full (may be NULL): Monte Carlo
 * evaluations per stage, repeated ones included; bracket_out (may be NULL):
 * the last bracket searched ([p, p] for an answer found by a single probe).
 * NT_ERR_NOT_BRACKETED when no bracket holds the target. */
nt_status nt_tolerable_rate_auto(nt_ctx *ctx, const nt_circuit *c, double P_target, double tol, uint64_t seed,
                                 uint64_t n_traj, double tau, double *p_star, int *n_coarse, int *n_full,
                                 double bracket_out[2]);

/* Tolerable uniform rate by the paper's steps (Sec. IV-D, Fig. 3), for the
 * fidelity criterion:
 *   1. exhaustive single-error simulation (nt_exhaustive): P_e per Pauli
 *      type, P_R of the error-free state;
 *   2. the success probability at one average error, by Eq. 4 with
 *      E(N_e) = 1/3 per type: P1 = (P_X + P_Y + P_Z) / 3;
 *   3. if P1 <= P_target, at most one error is tolerable and Eq. 5 gives the
 *      rate (nt_eq5 with the S error locations as units): *method = 0, no
 *      Monte Carlo run;
 *   4. otherwise Monte Carlo at increasing rates 2^k / S, k = 0, 1, ...
 *      (trajectories [0, n_traj), uniform model) while the success
 *      probability stays at or above P_target (by halves below 1/S when it
 *      is already under the target there); a rate within tol is the answer,
 *      else nt_tolerable_rate searches between the last two rates
 *      (the paper's Powell search, read as in nt_tolerable_rate):
 *      *method = 1.
 * n_probes (may be NULL): Monte Carlo evaluations, including the search's.
 * P_single (may be NULL): P_X, P_Y, P_Z, P_R from step 1.
 * NT_ERR_NOT_BRACKETED when P_R < P_target or no rate in [1e-9, 0.5]
 * brackets the target; NT_ERR_UNSUPPORTED for the measurement criteria. */
nt_status nt_tolerable_rate_fig3(nt_ctx *ctx, const nt_circuit *c, double P_target, double tol, uint64_t seed,
                                 uint64_t n_traj, double tau, double *p_star, int *method, int *n_probes,
                                 double P_single[4]);

/* Short-cuts for Monte Carlo runs.  ZERO_FIRED, CHECKPOINT and REUSE keep
 * every value bit-identical to the full run; LAST_ERROR is exact in
 * arithmetic only (see below):
 * NT_SHORTCUT_ZERO_FIRED -- a trajectory with no fired site ends in the
 *   error-free state, so its fidelity is 1 without simulating it (for the
 *   probability criteria: the error-free state's value, computed once);
 * NT_SHORTCUT_CHECKPOINT -- the error-free state before every pass is kept in
 *   device memory and a trajectory starts at the pass holding its first
 *   error (silently off when the checkpoints do not fit).
 * NT_SHORTCUT_LAST_ERROR -- a trajectory is scored right after the pass
 *   holding its last error, against the error-free state at that point: the
 *   rest of the circuit is one unitary applied to both states and leaves
 *   their overlap unchanged.  Exact in arithmetic only: fidelities differ
 *   from the full run by rounding, so a trajectory within rounding of tau
 *   can change sides and the success count can differ from the full run's
 *   (needs the checkpoints).  Not bit-identical, unlike the other three.
 * NT_SHORTCUT_REUSE -- a trajectory's criterion value is kept after it is
 *   simulated and reused by later runs of the same circuit, seed, precision,
 *   criterion and short-cut flags whose error model has the same Pauli-type
 *   proportions (p_x : p_y : p_z) -- e.g. the probes of nt_tolerable_rate or
 *   nt_sweep with the uniform model.  Rates are not part of the random draws
 *   (Sec. IV-B.2 sampling, common random numbers), so a trajectory's fired
 *   sets at any two rates are nested, and two rates with the same number of
 *   fired sites give it the same errors: (trajectory, count) identifies its
 *   value, which is reused bit for bit.  The store is emptied by every
 *   nt_set_shortcuts call, when any of the above changes, and when it
 *   exceeds 2^24 values.
 * Default 0 (every trajectory simulated in full). */
enum { NT_SHORTCUT_ZERO_FIRED = 1, NT_SHORTCUT_CHECKPOINT = 2, NT_SHORTCUT_LAST_ERROR = 4, NT_SHORTCUT_REUSE = 8 };
nt_status nt_set_shortcuts(nt_ctx *ctx, int flags);

/* ---- exhaustive single-error branch (Sec. IV-B.1, IV-C, IV-D) ---------------- */

/* Exhaustive Pauli error simulation (Sec. IV-B.1, Eq. 3): the circuit with
 * exactly one X, Y or Z error at each of its S sites (3S runs), scored by
 * the context's criterion.  fid_out (host, may be NULL): [S][3] criterion
 * values, columns X, Y, Z.  P_e[0..2]: success probability averaged over the
 * states with the same Pauli type (X, Y, Z); *P_R: success of the reference
 * state (Sec. IV-C). */
nt_status nt_exhaustive(nt_ctx *ctx, const nt_circuit *c, double tau, double *fid_out, double P_e[3],
                        double *P_R);

/* Eq. 4: P = sum_e P_e E_e + P_R (1 - sum_e E_e) for expected error counts
 * E_e (e = X, Y, Z).  Host arithmetic. */
nt_status nt_eq4(const double P_e[3], double P_R, const double E_e[3], double *P);

/* Eq. 5: tolerable uniform rate p = (1/units) (P - P_R) / (sum_e P_e/3 - P_R)
 * for target P; `units` is the number of error locations per circuit (the
 * paper writes G; the site count S makes Eq. 4 the first-order term of the
 * Monte Carlo model).  Host arithmetic; NT_ERR_INVALID_ARG if the
 * denominator is zero. */
nt_status nt_eq5(double P_target, const double P_e[3], double P_R, double units, double *p);

/* Success probability with the paper's method switch (Sec. IV-C, Fig. 2):
 * with E(N) = S (p_x + p_y + p_z) <= 1 expected errors, exhaustive
 * simulation and Eq. 4 (E_e = S p_e); otherwise Monte Carlo over trajectories
 * [0, n_traj).  *method: 0 = exhaustive + Eq. 4, 1 = Monte Carlo. */
nt_status nt_success_probability(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t n_traj, double tau,
                                 double *P, int *method);

/* ---- learned surrogate of the success curve ---------------------------------- */

/* A graph neural network over a circuit's gate graph predicts the success
 * probability (fidelity criterion) at the 13 rates 10^(-5 + j/4), j = 0..12,
 * trained on Monte Carlo labels; the tolerable-rate search uses it to bracket
 * the rate (the Monte Carlo search then runs inside the bracket, with the
 * full bracket as fallback, so the surrogate never decides the result).
 * Graph: one node per gate, an edge between consecutive gates on a qubit.
 * Node features (32): one-hot kind (17), sin/cos of up to three angles (6),
 * ASAP layer / depth, arity - 1, n / 16, 1, zero padding.  Globals: n / 16,
 * G / 2048, S / 4096, 1.  Network: input layer 32 -> 64 (ReLU); 3 layers
 * H' = ReLU(H Ws + mean_nbr(H) Wn + b); mean pool; [pool, globals] (68) ->
 * 64 (ReLU) -> 13 (sigmoid); loss: mean squared error.  Dense products use
 * bf16 MFMA with FP32 accumulation ("exact" = 0) or plain FP32 ("exact" = 1,
 * for gradient checks).  Deterministic: fixed-order reductions, no
 * floating-point atomics.  One model per context; the model uses the
 * context's device and stream. */
typedef struct nt_gnn nt_gnn;
nt_status nt_gnn_create(nt_ctx *ctx, uint64_t seed, nt_gnn **out);
void nt_gnn_destroy(nt_gnn *m);
/* Host-only graph of a circuit.  Pass NULL buffers to query the sizes:
 * *n_nodes = G, *n_edges = entries of col.  x: [n_nodes][32], row_ptr:
 * [n_nodes + 1], col: neighbour indices, glob: [4]. */
nt_status nt_gnn_graph(const nt_circuit *c, float *x, int32_t *row_ptr, int32_t *col, float *glob, int64_t *n_nodes,
                       int64_t *n_edges);
/* Flat parameter vector (FP32): W_in [32][64], b_in [64]; per layer
 * Ws [64][64], Wn [64][64], b [64]; W_h1 [68][64], b_h1 [64]; W_h2 [64][13],
 * b_h2 [13] (row-major, input index first).  out NULL: *len = size. */
nt_status nt_gnn_params(nt_gnn *m, float *out, int64_t *len);
nt_status nt_gnn_set_params(nt_gnn *m, const float *in, int64_t len);
/* Training set: circuits and labels [n][13] (host; NULL for none). */
nt_status nt_gnn_set_data(nt_gnn *m, const nt_circuit *const *circuits, int n, const float *labels);
/* Loss and gradient (host, length of the parameter vector) over training
 * graphs [g0, g1). */
nt_status nt_gnn_loss_grad(nt_gnn *m, int g0, int g1, int exact, double *loss, float *grad);
/* Adam (beta 0.9 / 0.999, eps 1e-8) over mini-batches of batch_graphs
 * consecutive graphs, batch order shuffled per epoch (seeded);
 * loss_out[epochs] (host, may be NULL): mean training loss per epoch. */
nt_status nt_gnn_train(nt_gnn *m, int epochs, int batch_graphs, double lr, uint64_t seed, double *loss_out);
/* Predicted success probabilities, out [n][13] (host). */
nt_status nt_gnn_predict(nt_gnn *m, const nt_circuit *const *circuits, int n, int exact, float *out);

/* Tolerable rate guided by the surrogate (an accelerator of the search of
 * Sec. IV-D, not part of the paper).  From the predicted curve, the rate p^
 * where it crosses P_target (linear in log10 p between the two grid points
 * around the crossing).  One Monte Carlo probe at p^; if it is within tol of
 * P_target, p^ is the answer.  Otherwise nt_tolerable_rate in half a grid
 * step (a factor 10^(1/8)) from p^ on the side the probe points to, then in
 * the grid interval of the crossing widened by one grid step per side, then
 * over the whole grid [1e-5, 1e-2]; when the prediction does not cross
 * P_target, the whole grid directly.  With NT_SHORTCUT_REUSE on, rates probed
 * again cost no simulation.  bracket_out (may be NULL): the bracket the
 * search ended in ([p^, p^] after a one-probe answer).  *n_probes counts
 * every Monte Carlo evaluation, repeated ones included. */
nt_status nt_tolerable_rate_guided(nt_ctx *ctx, const nt_circuit *c, nt_gnn *m, double P_target, double tol,
                                   uint64_t seed, uint64_t n_traj, double tau, double *p_star, int *n_probes,
                                   double bracket_out[2]);

/* ---- parity and debug exports ---------------------------------------------- */

/* Fired error sites of trajectories [traj_begin, traj_begin + n_traj) under
 * the current error model, drawn on the device: CSR with offsets[n_traj+1]
 * (host), sites (site index) and paulis (1 = X, 2 = Y, 3 = Z), in site order.
 * cap = capacity of sites/paulis; NT_ERR_BUFFER_TOO_SMALL with the required
 * total in *n_out when it is too small (offsets are still filled). */
nt_status nt_sample_sites(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t traj_begin,
                          uint64_t n_traj, uint64_t *offsets, int32_t *sites, uint8_t *paulis,
                          int64_t cap, int64_t *n_out);

/* Final amplitudes of trajectory `traj` (current error model and precision).
 * amps_out: host or device, len = 2^n amplitudes in the current precision. */
nt_status nt_final_state(nt_ctx *ctx, const nt_circuit *c, uint64_t seed, uint64_t traj,
                         void *amps_out, int64_t len);

/* Error-free final state (the reference of the fidelity criterion). */
nt_status nt_reference_state(nt_ctx *ctx, const nt_circuit *c, void *amps_out, int64_t len);

/* ---- timing (HIP events on the context stream) ------------------------------ */

/* When enabled, every gate-pass kernel launch is bracketed by HIP events on
 * the context stream.  nt_timing_read returns, since the last reset, the
 * number of pass launches, their summed duration (ms), their summed
 * algorithmic HBM bytes (each pass reads and writes every state once; the
 * first pass only writes; the scoring pass reads the state and the
 * reference), amplitude-updates (gates x amplitudes x trajectories) and
 * algorithmic floating-point operations, counted per gate of the circuit
 * whatever ops the plan fuses them into (per amplitude: a permutation with
 * unit phases such as X, Y, CNOT or SWAP 0; a diagonal 6 per entry other
 * than 1, averaged over the amplitudes, so RZ and RZZ 6, Z, S and T 3, CZ
 * and CP 1.5; any other one-qubit gate 14, two-qubit gate 30; the fused
 * scoring 8).  Reading synchronizes the stream. */
nt_status nt_timing_enable(nt_ctx *ctx, int enable);
nt_status nt_timing_reset(nt_ctx *ctx);
nt_status nt_timing_read(nt_ctx *ctx, int64_t *n_launches, double *ms_total, double *bytes_total,
                         double *updates_total, double *flops_total);

/* Thread-local text of the last failure ("" if none). */
const char *nt_last_error(void);

/* Library version string. */
const char *nt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NISQTOL_H */
