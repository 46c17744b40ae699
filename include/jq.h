/*
 * jq - state-vector gate application on one MI355X (gfx950).
 *
 * The operations follow De Raedt et al., "Massively parallel quantum computer
 * simulator, eleven years later" (Comput. Phys. Commun.):
 *
 *  - the state of N qubits is a vector of 2^N complex amplitudes (Sec. 2,
 *    Eq. STAT2); qubit j is bit j of the basis index, qubit 0 the least
 *    significant bit;
 *  - a circuit is a sequence of unitary operations on that vector (Sec. 2);
 *    a single-qubit gate updates 2^(N-1) amplitude pairs in place (Eq. NUM2),
 *    a two-qubit gate 2^(N-2) groups of four (Sec. 2);
 *  - outputs are the amplitudes and the outcome probabilities of qubits
 *    (Sec. 2, last paragraph);
 *  - three encodings: complex128 (the E flavour, 16 B per amplitude, Sec. 1),
 *    complex64 (8 B), and the adaptive two-byte polar code of Sec. 4.1.
 *
 * Conventions that hold for every call:
 *  - Every call returns an int: JQ_OK (0) or a negative error code, and on
 *    error jq_last_error() (thread-local) describes it.  Arguments are
 *    checked on the host before anything is enqueued; on an argument error
 *    the state is unchanged.  A device fault surfaces as JQ_EDEVICE at the
 *    next call that synchronises.
 *  - Pointers named "host" below are host memory owned by the caller and
 *    only read or written during the call.  Device memory of a state is
 *    owned by the library (allocated through the registered allocator, see
 *    jq_set_allocator, else hipMalloc) and freed by jq_state_destroy.
 *  - Calls that only enqueue work are asynchronous on the state's stream;
 *    calls that return data (norm, probabilities, read) synchronise it.
 *  - Complex numbers on the host are interleaved (re, im) doubles.
 *  - Matrices are row-major; for a two-qubit gate the first listed qubit is
 *    the most significant bit of the row/column index, the basis
 *    |control,target> that App. A uses for CNOT and U(k).  Outputs of
 *    jq_probabilities use the opposite, state-like order: bit m of the
 *    output index is the value of qubits[m].
 *  - A jq_state must not be used from two threads at once.
 */
#ifndef JQ_H
#define JQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define JQ_OK 0
#define JQ_EINVAL (-1)       /* invalid argument */
#define JQ_ENOMEM (-2)       /* not enough device (HBM) memory */
#define JQ_EDEVICE (-3)      /* HIP runtime error or device fault */
#define JQ_EUNSUPPORTED (-4) /* a valid request the library does not implement */
#define JQ_EZERO (-5)        /* projection onto a zero-probability outcome */
#define JQ_EBUSY (-6)        /* server queue full (non-blocking submit) */

#define JQ_MAX_QUBITS 63
#define JQ_MAX_CONTROLS 4

/* Amplitude encodings (Sec. 1: E = complex128; Sec. 4.1: the two-byte
 * code, stored as two int8 planes b0[2^N] then b1[2^N] plus the FP64
 * range (r0, r1) in device memory). */
typedef enum { JQ_C128 = 0, JQ_C64 = 1, JQ_COMPACT = 2 } jq_encoding;

/* Initial states: |0...0> (Sec. 2), the uniform superposition 2^(-N/2)
 * (Sec. 5.1), or a basis state |basis>. */
typedef enum { JQ_INIT_ZERO = 0, JQ_INIT_UNIFORM = 1, JQ_INIT_BASIS = 2 } jq_init;

/* Gate classes.  DENSE: a full 2^nq x 2^nq matrix.  DIAGONAL: only the
 * 2^nq diagonal entries are given.  PERM_X: the bit flip X of App. A on one
 * target (with controls this is CNOT or TOFFOLI); no matrix. */
typedef enum { JQ_DENSE = 0, JQ_DIAGONAL = 1, JQ_PERM_X = 2 } jq_gate_kind;

/* Quantisation of the two-byte code.  PER_GATE decodes and re-encodes the
 * state around every gate, recomputing (r0, r1) each time (Sec. 4.1 as the
 * paper runs it).  PER_BLOCK does so once per fused block of gates. */
typedef enum { JQ_COMPACT_PER_GATE = 0, JQ_COMPACT_PER_BLOCK = 1 } jq_compact_mode;

/* One gate.  qubits[0..nq-1] are the targets (nq = 1 or 2; nq = 1 for
 * PERM_X), controls[0..nc-1] the controls (all must be 1 for the gate to
 * act).  m holds the matrix: 2^nq x 2^nq row-major complex for DENSE, the
 * 2^nq diagonal entries for DIAGONAL, unused for PERM_X.  All qubits of a
 * gate must be distinct and in [0, N). */
typedef struct {
    int32_t kind;
    int32_t nq;
    int32_t nc;
    int32_t qubits[2];
    int32_t controls[JQ_MAX_CONTROLS];
    int32_t pad_;
    double m[32];
} jq_gate;

/* Execution options for jq_apply_circuit (NULL = defaults).
 *  fusion:      0 = let the planner fuse gates into register-blocked tile
 *               passes with its tuned width; 1 = one kernel per gate;
 *               k >= 2 = fuse with at most k register qubits per pass.
 *  compact_mode: a jq_compact_mode, used for JQ_COMPACT states.  In
 *               PER_BLOCK mode a block is one fused pass (or one gate
 *               the planner leaves unfused); JQ_EINVAL for other values.
 *  max_ops:     upper bound on gates per fused pass (0 = default).
 *  search:      the planner's large-state steps (a search over which qubits
 *               take a pass's tile slots, the choice of register vs lane
 *               slot for each of them, and the order of the lane bits):
 *               JQ_SEARCH_AUTO (0) = on for states of 1 GiB or more, off
 *               below; JQ_SEARCH_ON = on at any size; JQ_SEARCH_OFF = off
 *               at any size; JQ_EINVAL for other values.  The result is
 *               the same either way up to floating-point rounding; the
 *               switch exists so that small states can run the plans
 *               large states get.
 *  reserved:    must be zero.
 * jq_plan_schedule reports the blocks a circuit will run as. */
#define JQ_SEARCH_AUTO 0
#define JQ_SEARCH_ON 1
#define JQ_SEARCH_OFF 2
typedef struct {
    int32_t fusion;
    int32_t compact_mode;
    int32_t max_ops;
    int32_t search;
    int32_t reserved[4];
} jq_exec_opts;

/* Tuning of the single-state path for one device, encoding and state size.
 * The paper proposes combining gates into multi-qubit blocks to raise the
 * work per byte moved (Sec. 5.2) but gives no rule for how; these are the
 * choices the planner and the per-gate kernels make, and jq_autotune picks
 * them by timing them on the device:
 *  k_reg:       register bits of a fused tile pass (a lane holds 2^k_reg
 *               amplitudes): 2..5 for JQ_C128, 2..6 for JQ_C64.  Unless
 *               every gate of the circuit is an uncontrolled one-qubit
 *               dense gate or a controlled Z, the planner uses at most 4
 *               (JQ_C128) or 5 (JQ_C64), the widest at which the fused
 *               kernel for the other op kinds keeps 4 waves per SIMD; a
 *               width given in opts->fusion is used as given;
 *  pass_ops:    the planner's weight of one more pass against one more op
 *               in a pass (a pass's streaming time in units of one fused
 *               op's arithmetic), in (0, 10000];
 *  wide_mask:   per-gate dense and X kernels take four amplitude pairs per
 *               thread for each target whose bit is set, one pair for the
 *               others (which is faster depends on the target's stride and
 *               the device's address interleave: jq_autotune times both on
 *               every target);
 *  wide_target: the same choice as a threshold, for jq_tuning_set: with
 *               wide_mask = 0 the targets from wide_target up (0..64; 64:
 *               none) take four pairs.  jq_tuning_get reports the lowest
 *               target in wide_mask (64: none);
 *  search:      the planner's large-state steps (see jq_exec_opts.search):
 *               JQ_SEARCH_AUTO (on from 1 GiB of state up), JQ_SEARCH_ON or
 *               JQ_SEARCH_OFF; an explicit opts->search wins;
 *  n_qubits:    the state size the values were tuned at (0: the built-in
 *               defaults);
 *  source:      JQ_TUNE_DEFAULT, JQ_TUNE_MEASURED (jq_autotune in this
 *               process), JQ_TUNE_CACHED (read from the cache file) or
 *               JQ_TUNE_SET (jq_tuning_set);
 *  tuned_ms, default_ms: jq_autotune's time of its tuning circuit with the
 *               chosen values and with the built-in defaults (0 otherwise).
 * jq_apply_circuit (and the request loop) use the values for the state's
 * device, encoding and N when opts is NULL or opts->fusion is 0: an entry
 * for exactly N, else, for N >= 25 (states past the last-level cache), the
 * entry of the largest tuned size from 25 up to N, else the defaults.  The
 * two-byte code is not tuned.  Plans depend only on (circuit, N, encoding,
 * tuning), so a result is the same alone and in a mix as long as the tuning
 * does not change in between. */
#define JQ_TUNE_DEFAULT 0
#define JQ_TUNE_MEASURED 1
#define JQ_TUNE_CACHED 2
#define JQ_TUNE_SET 3
typedef struct {
    int32_t k_reg;
    int32_t wide_target;
    double pass_ops;
    int32_t n_qubits;
    int32_t source;
    double tuned_ms;
    double default_ms;
    int32_t search;
    int32_t reserved_;
    uint64_t wide_mask;
} jq_tuning;

/* The tuning jq_apply_circuit uses for an N-qubit state of encoding enc on
 * the current device (host only; with no GPU visible the device is taken as
 * "host").  The first call in a process reads the cache file: the path in
 * the environment variable JQ_TUNE_CACHE, else $HOME/.cache/jq/tuning.json
 * (a missing or unreadable file counts as empty).  JQ_EINVAL for a bad N or
 * encoding. */
int jq_tuning_get(int n_qubits, int enc, jq_tuning *out);

/* Set the tuning for N-qubit states of encoding enc on the current device
 * for the rest of the process (host only; nothing is written to the cache
 * file); t = NULL removes a value set before.  JQ_EINVAL if a field is out
 * of range (the table is then unchanged) or enc is JQ_COMPACT. */
int jq_tuning_set(int n_qubits, int enc, const jq_tuning *t);

/* Measure the tuning for N-qubit states of encoding enc (JQ_C128 or JQ_C64,
 * 10 <= N <= 34) on the current device: a scratch state of 2^N amplitudes
 * runs a tuning circuit under each register width from 3 up and three
 * planner weights, and the fastest set is kept if it beats the defaults
 * (among those timed) by 2% or more; the large-state steps are then timed
 * switched the other way than the size rule has them, and kept that way
 * under the same 2% rule; a dense gate on every target from 8 up is timed
 * with one and with four pairs per thread, and a target takes four where
 * that is 2% faster or more (the targets below 8, and from N up, keep the
 * default and the highest timed target's choice).  The tuning circuit is gates[0..count-1]
 * (the caller's workload, validated as by jq_apply_circuit; the best
 * register width depends on a circuit's depth and structure), or, with
 * count = 0, ten layers of random U(2) on every qubit and CZ on a random
 * matching.  The cache file holds one entry per device, encoding and N:
 * the last tuning.  The result is kept for the
 * process and merged into the cache file.  flags: JQ_TUNE_FORCE measures
 * even when the cache file has an entry for this device, encoding and N
 * (otherwise that entry is returned); JQ_TUNE_NO_CACHE neither reads nor
 * writes the file.  JQ_ENOMEM if the scratch state does not fit; the
 * device memory of the scratch state is freed before return.  Synchronous. */
#define JQ_TUNE_FORCE 1
#define JQ_TUNE_NO_CACHE 2
int jq_autotune(int n_qubits, int enc, int flags, const jq_gate *gates, size_t count, jq_tuning *out);

typedef struct jq_state jq_state;

/* ---- state lifetime -------------------------------------------------- */

/* Create an N-qubit state (1 <= N <= JQ_MAX_QUBITS; App. A, QUBITS) in the
 * given encoding on the current HIP device, initialised to |0...0>.
 * 2^N * bytes-per-amplitude (16, 8, 2) must fit in free device memory, else
 * JQ_ENOMEM.  *out receives the handle. */
int jq_state_create(int n_qubits, jq_encoding enc, jq_state **out);

/* Free the state's device memory; the handle is invalid afterwards. */
int jq_state_destroy(jq_state *s);

/* Set the state to |0...0>, the uniform superposition, or |basis>
 * (basis < 2^N).  Asynchronous. */
int jq_state_init(jq_state *s, jq_init mode, uint64_t basis);

/* Set the state to the SHORBOX state of App. A (Sec. 5.3):
 * 2^(-n_x/2) sum over x = 0 .. 2^n_x - 1 of |x>|y^x mod G>, the x-register
 * on qubits 0 .. n_x-1 (x's least significant bit on qubit 0) and the
 * f-register on the qubits above.  Needs 1 <= n_x < N, n_x <= 40,
 * 2 <= G < 2^32, G <= 2^(N - n_x) and 1 < y < G (y coprime to G for
 * Shor's algorithm; not checked), else JQ_EINVAL.  Asynchronous. */
int jq_shorbox(jq_state *s, int n_x, uint64_t G, uint64_t y);

/* Number of qubits, encoding, and device bytes held (host outputs; any may
 * be NULL). */
int jq_state_info(const jq_state *s, int *n_qubits, int *encoding, uint64_t *bytes);

/* Device address of the amplitude storage (for c128/c64: 2^N interleaved
 * complex values; for compact: the b0 plane followed by the b1 plane). */
int jq_state_device_ptr(const jq_state *s, void **ptr);

/* Run the state's work on this hipStream_t (NULL = the library's own
 * stream).  The stream must outlive its use by the state. */
int jq_set_stream(jq_state *s, void *hip_stream);

/* Wait until all work enqueued for the state has finished. */
int jq_synchronize(jq_state *s);

/* Route state allocations through alloc(bytes, ctx) / release(ptr, ctx)
 * (for example a framework's caching allocator).  Both NULL restores
 * hipMalloc/hipFree.  States keep the functions they were created with. */
int jq_set_allocator(void *(*alloc)(size_t, void *), void (*release)(void *, void *), void *ctx);

/* ---- gates ----------------------------------------------------------- */

/* Lower a named instruction of App. A into a jq_gate (host only, no
 * device work).  Names: I H X Y Z S S+ T T+ U1 U2 U3 +X -X +Y -Y R CNOT U
 * TOFFOLI, plus RZ (diag(e^{-i t/2}, e^{i t/2})), CZ (= U with k=1),
 * CP (diag(1,1,1,e^{i phi})), SWAP, MAT1 (8 params: explicit 2x2) and
 * MAT2 (32 params: explicit 4x4).  qubits as in App. A's syntax (controls
 * first); params are the angles or k of App. A.  Returns JQ_EINVAL on an
 * unknown name or wrong argument count.  "I" lowers to an empty gate
 * (nq = 0) that jq_apply_circuit skips. */
int jq_gate_named(const char *name, const int *qubits, int nq, const double *params, int np, jq_gate *out);

/* Lower count named instructions in one call: jq_gate_named on each, then
 * instruction i's extra controls appended to its record (after the
 * controls its name implies).  names[i] is instruction i's name; nq[i],
 * np[i] and nc[i] count its qubits, parameters and extra controls, whose
 * values follow one another, instruction by instruction, in qubits, params
 * and controls (each may be NULL when its counts are all zero; nc itself
 * may be NULL: no extra controls).  out holds count records.  Host only.
 * Returns JQ_OK, or JQ_EINVAL for the first bad instruction (its index in
 * jq_last_error; the records before it are filled) or for more than
 * JQ_MAX_CONTROLS controls in one record. */
int jq_gates_named(size_t count, const char *const *names, const int *nq, const int *qubits, const int *np,
                   const double *params, const int *nc, const int *controls, jq_gate *out);

/* Apply one gate (Sec. 2, Eq. NUM2 and its four-amplitude analogue).
 * matrix is copied before return.  JQ_EINVAL if the qubits are invalid or
 * the matrix does not fit the kind (e.g. a non-zero off-diagonal entry for
 * DIAGONAL).  Asynchronous. */
int jq_apply_gate(jq_state *s, int kind, const int *qubits, int nq, const int *controls, int nc,
                  const double *matrix);

/* Apply gates[0..count-1] in order.  All gates are validated first; on an
 * invalid gate nothing is applied.  Gates may be fused into tile passes
 * (see jq_exec_opts); the result equals applying them one by one up to
 * floating-point rounding.  Asynchronous. */
int jq_apply_circuit(jq_state *s, const jq_gate *gates, size_t count, const jq_exec_opts *opts);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * jq_apply_circuit, with the same validation, plan, kernels and results
 * (bit for bit), except that the plan's fused-op list is staged in a fixed
 * device workspace of JQ_NOALLOC_WORKSPACE_BYTES per GPU (held until the
 * process ends) instead of per-state buffers, and per-launch timing
 * (jq_profile_enable) is not recorded.  It calls no hipMalloc, hipFree or
 * other allocating routine; the state's device must be current.
 * JQ_EINVAL, with nothing enqueued and the state unchanged, if the plan has
 * more fused ops than the workspace holds (jq_plan_steps gives the plan; a
 * fused op takes 704 bytes, so about 5900 fit).  Every call on one GPU
 * shares that GPU's workspace, which keeps the last call's ops: calls on one
 * stream are ordered, but calls whose work overlaps on one GPU (other
 * streams without synchronisation between them, concurrent threads) race,
 * and the caller must serialise them.  Asynchronous. */
#define JQ_NOALLOC_WORKSPACE_BYTES (4u << 20)
int jq_apply_circuit_noalloc(jq_state *s, const jq_gate *gates, size_t count, const jq_exec_opts *opts);

/* jq_apply_circuit with the depolarizing channel of App. A: after each gate
 * (identity gates included), every qubit q receives an X gate with
 * probability px, a Y gate with probability py or a Z gate with probability
 * pz, decided by the caller's draw u[g * N + q] in [0, 1) for gate g: X if
 * u < px, Y if px <= u < px + py, Z if px + py <= u < px + py + pz, no gate
 * otherwise.  u holds count * N draws (host; the library draws no random
 * numbers).  JQ_EINVAL unless px, py, pz >= 0 with px + py + pz <= 1 and
 * every draw lies in [0, 1); the state is unchanged on error.  The
 * inserted gates are planned and fused with the circuit.  Asynchronous. */
int jq_apply_circuit_noisy(jq_state *s, const jq_gate *gates, size_t count, double px, double py, double pz,
                           const double *u, const jq_exec_opts *opts);

/* The schedule jq_apply_circuit follows for these gates on an N-qubit state
 * of encoding enc with these options (host only: no device work, no state).
 * The planner groups gates into blocks (Sec. 5.2 proposes such fusion); a
 * gate may move ahead of earlier gates it commutes with (they share no
 * qubit, or both are diagonal).  order[0..k-1] receives the input index of
 * each non-identity gate in the order applied (inside a fused block, gates
 * that commute with everything between may run at another point of the
 * block: the product is the same); block_len[0..*n_blocks-1]
 * the number of gates of each consecutive block of that order, and
 * block_fused[b] (may be NULL) 1 for a fused tile pass, 0 for a single-gate
 * kernel.  order, block_len and block_fused need room for count entries.
 * For JQ_COMPACT in PER_BLOCK mode each block is decoded and encoded once.
 * Validation and errors as jq_apply_circuit. */
int jq_plan_schedule(int n_qubits, int enc, const jq_gate *gates, size_t count, const jq_exec_opts *opts,
                     int32_t *order, int32_t *block_len, int32_t *block_fused, size_t *n_blocks);

/* One step of the plan of jq_plan_schedule, as the kernels see it. */
typedef struct {
    int32_t fused;     /* 1: a fused tile pass (Sec. 5.2's combined gates), 0: one gate alone */
    int32_t k_reg;     /* register bits of the pass: a lane holds 2^k_reg amplitudes */
    int32_t reg_q[8];  /* qubit held by register slot j (j < k_reg), else -1 */
    int32_t lane_q[6]; /* qubit held by lane bit b */
    int32_t n_gates;   /* source gates of the step */
    int32_t n_ops;     /* kernel ops of the pass after folding and merging */
    int32_t table_tag; /* element type of the pass's per-slot diagonal tables:
                          0 none, 1 FP64 pairs (at most 16 slots), 2 FP32 pairs
                          (at most 32 slots); always the fused kernel's type */
    int32_t n_tables;  /* ops of the pass that carry such a table */
} jq_plan_step;

/* The steps jq_apply_circuit runs for these gates (host only, no device
 * work): out[0..min(max, *n_steps)-1] receives them (out may be NULL with
 * max = 0 to count).  Validation and errors as jq_plan_schedule. */
int jq_plan_steps(int n_qubits, int enc, const jq_gate *gates, size_t count, const jq_exec_opts *opts,
                  jq_plan_step *out, size_t max, size_t *n_steps);

/* ---- reductions (FP64 whatever the encoding) ------------------------ */

/* Squared norm sum |a_i|^2 (the left side of Eq. STAT1).  Synchronises. */
int jq_norm(jq_state *s, double *out);

/* Marginal distribution over qubits[0..nq-1] (distinct, 0 <= nq <= N,
 * nq <= 30): out (host, 2^nq doubles) receives sum |a_i|^2 over the basis
 * states whose bit qubits[m] equals bit m of the output index (Sec. 2).
 * Deterministic summation order.  Synchronises. */
int jq_probabilities(jq_state *s, const int *qubits, int nq, double *out);

/* Expectation values <Qx(n)>, <Qy(n)>, <Qz(n)> = <(1 - sigma^alpha_n)>/2 of
 * every qubit (App. A, BEGIN MEASUREMENT); qx, qy, qz are host arrays of N
 * doubles (any may be NULL).  Synchronises. */
int jq_expectations(jq_state *s, double *qx, double *qy, double *qz);

/* Scale the state to unit norm, in FP64.  For the two-byte code this scales
 * (r0, r1) and leaves the codes alone.  JQ_EZERO if the norm is zero. */
int jq_renormalize(jq_state *s);

/* Draw basis states from the distribution |a_i|^2 (App. A, GENERATE
 * EVENTS), leaving the state unchanged.  u[0..count-1] (host) are draws in
 * [0, 1) the caller supplies (the library draws no random numbers); out[k]
 * (host) receives the least i whose cumulative probability (FP64, summed in
 * index order in fixed blocks) exceeds u[k] times the total.  Indices of
 * zero probability are never returned.  JQ_EINVAL for a draw outside
 * [0, 1), JQ_EZERO for a zero state.  Synchronises. */
int jq_sample(jq_state *s, const double *u, size_t count, uint64_t *out);

/* ---- auxiliary-variable amplitudes (Sec. 4.2) ------------------------- */

/* Amplitudes <b|psi> of psi = gates applied to |0...0> on N qubits
 * (1 <= N <= 63), computed without a state vector by the auxiliary-variable
 * method of Sec. 4.2 (Eqs. appa2-appa7): every controlled phase shift
 * (CZ, U(k), CP, a two-qubit diagonal, a singly controlled one-qubit
 * diagonal) and every CNOT (as H U(pi) H on its target) gets a two-valued
 * variable; for each of the 2^P assignments the qubits evolve one by one,
 * and the amplitude is 2^-P times the sum over assignments of the product
 * of the qubits' components (FP64).  Time O(2^P (G + N M)), memory O(N + M).
 * Supported: one-qubit gates without controls, X with at most one control,
 * diagonal gates as listed; anything else (Toffoli, SWAP, MAT2, controlled
 * dense gates) returns JQ_EUNSUPPORTED, as do more than 40 entangling
 * gates.  basis[0..m-1] (host) are indices below 2^N; out (host) receives
 * m interleaved complex values.  Runs on the current HIP device and
 * allocates its own small buffers.  Synchronises. */
int jq_aux_amplitudes(int n_qubits, const jq_gate *gates, size_t count, const uint64_t *basis, size_t m,
                      double *out);

/* ---- projection (App. A: CLEAR, SET, M) ------------------------------- */

/* Project qubit `qubit` onto |value> (value 0: CLEAR, 1: SET) and
 * renormalise: p = sum of |a_i|^2 over the basis states whose bit `qubit`
 * equals value (FP64, as jq_probabilities); those amplitudes are divided by
 * sqrt(p), all others become zero.  *p_out (may be NULL) receives p.
 * JQ_EZERO if p is zero: the projection would leave no amplitude (the
 * paper's instructions fail then) and the state is unchanged.  For the
 * two-byte code the projection is one quantisation step with a new range.
 * Synchronises (p decides what runs). */
int jq_project(jq_state *s, int qubit, int value, double *p_out);

/* Projective measurement of qubit `qubit` (App. A, M).  p0 and p1 are the
 * FP64 probabilities of the two outcomes; the outcome is 1 when
 * u >= p0 / (p0 + p1), else 0, where u in [0, 1) is a random number the
 * caller draws (the library draws none); the state is then projected onto
 * the outcome as by jq_project.  *outcome receives 0 or 1 and *p1_out (may
 * be NULL) p1 / (p0 + p1).  JQ_EINVAL if u is outside [0, 1) or outcome is
 * NULL, JQ_EZERO if the state is zero.  Synchronises. */
int jq_measure(jq_state *s, int qubit, double u, int *outcome, double *p1_out);

/* ---- amplitude transfer --------------------------------------------- */

/* Copy amplitudes [first, first+count) to host as complex128 (decoded for
 * the two-byte code).  Synchronises. */
int jq_read_amplitudes(jq_state *s, uint64_t first, uint64_t count, double *out);

/* Overwrite amplitudes [first, first+count) from host complex128.  For the
 * two-byte code only a full write (first = 0, count = 2^N) is allowed; it
 * takes (r0, r1) from the data as the encoder does.  Synchronises. */
int jq_write_amplitudes(jq_state *s, uint64_t first, uint64_t count, const double *in);

/* Two-byte code only: copy codes [first, first+count) of both planes to
 * host int8 arrays (either may be NULL) and the current range to range[2]
 * (may be NULL).  Synchronises. */
int jq_read_codes(jq_state *s, uint64_t first, uint64_t count, int8_t *b0, int8_t *b1, double *range);

/* Two-byte code only: overwrite all 2^N codes of both planes from host int8
 * arrays and set the range to range[2] = (r0, r1), 0 <= r0 <= r1 (used
 * for restoring a saved state).  A zero modulus code (-128) must carry phase
 * code 0.  Synchronises. */
int jq_write_codes(jq_state *s, const int8_t *b0, const int8_t *b1, const double *range);

/* ---- per-launch timing ------------------------------------------------ */

typedef struct {
    char name[32];    /* kernel class */
    uint64_t launches;
    double total_ms;  /* sum of hipEvent-measured launch durations */
    double bytes;     /* algorithmic HBM bytes of those launches */
} jq_kernel_stat;

/* Record a hipEvent pair on the state's stream around every kernel launch
 * (on != 0) or stop (on == 0); enabling clears the counters. */
int jq_profile_enable(jq_state *s, int on);

/* Synchronise and report per-class totals; writes up to max entries and
 * the number of classes to *count. */
int jq_profile_read(jq_state *s, jq_kernel_stat *out, int max, int *count);

/* ---- batched small circuits ---------------------------------------- */

/* A circuit for batch or serving use: n_qubits and gates[0..n_gates-1]
 * (host memory, read during the call that takes it). */
typedef struct {
    int32_t n_qubits;
    int32_t pad_;
    uint64_t n_gates;
    const jq_gate *gates;
} jq_circuit;

typedef struct jq_batch jq_batch;

/* Prepare count independent circuits (each 1 <= N <= 20) for one
 * persistent launch: gates are lowered and packed into device memory and a
 * packed state arena is allocated.  enc is JQ_C128 or JQ_C64.  Work runs on
 * hip_stream (NULL = the library's stream).  opts->fusion sets the fusion
 * depth of every circuit: 1..3 = blocks of consecutive gates on at most that
 * many target qubits; 4 = register/lane tile passes (as for a single large
 * state) for states too large for LDS, blocks of 3 for the others; 0 or
 * opts NULL = chosen per (encoding, N) by timing on first use in the
 * process. */
int jq_batch_create(const jq_circuit *circuits, size_t count, jq_encoding enc, const jq_exec_opts *opts,
                    void *hip_stream, jq_batch **out);

/* Reset every state to |0...0> and run every circuit, in one kernel launch
 * (a persistent grid that pulls circuits from a device work counter).
 * Asynchronous; elapsed_ms (may be NULL) receives the launch's
 * hipEvent-measured time after synchronising when non-NULL. */
int jq_batch_run(jq_batch *b, double *elapsed_ms);

/* Copy amplitudes of circuit `index` to host complex128.  Synchronises. */
int jq_batch_read(jq_batch *b, size_t index, uint64_t first, uint64_t count, double *out);

int jq_batch_destroy(jq_batch *b);

/* ---- serving ---------------------------------------------------------- */

typedef struct jq_server jq_server;

typedef struct {
    uint64_t ticket;
    int32_t status;        /* JQ_OK or the error of that request */
    int32_t n_qubits;
    double norm;           /* FP64 squared norm of the final state */
    double latency_ms;     /* submit -> device completion */
    double queue_ms;       /* submit -> admission */
    jq_state *state;       /* final state, resident until jq_server_release */
} jq_result;

typedef struct {
    uint64_t submitted, completed, rejected;
    double p50_ms, p99_ms, mean_ms;
    double throughput_per_s; /* completions / (last completion - first submit) */
    uint64_t peak_resident_bytes;
} jq_server_stats;

/* Start a request loop on the current device: admitted requests' states
 * may together hold at most hbm_budget bytes; work is spread over
 * n_streams streams; at most queue_cap requests wait for admission. */
int jq_server_create(uint64_t hbm_budget, int n_streams, int queue_cap, jq_encoding enc, jq_server **out);

/* Queue a circuit (copied).  blocking = 0 returns JQ_EBUSY when the queue
 * is full; a request whose state alone exceeds the budget is rejected with
 * JQ_ENOMEM.  *ticket identifies the request. */
int jq_server_submit(jq_server *sv, const jq_circuit *c, int blocking, uint64_t *ticket);

/* Wait for (timeout_ms < 0: forever) or poll (timeout_ms = 0) any finished
 * request; JQ_EBUSY if none finished in time.  The result's state stays
 * resident (and counts against the budget) until jq_server_release. */
int jq_server_wait(jq_server *sv, int timeout_ms, jq_result *out);

int jq_server_release(jq_server *sv, uint64_t ticket);
int jq_server_stats_get(jq_server *sv, jq_server_stats *out);
int jq_server_destroy(jq_server *sv);

/* ---- errors ----------------------------------------------------------- */

/* Description of the last error on this thread ("" if none). */
const char *jq_last_error(void);

/* Library version string. */
const char *jq_version(void);

#ifdef __cplusplus
}
#endif

#endif /* JQ_H */
