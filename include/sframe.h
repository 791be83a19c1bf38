/*
 * sframe -- stabilizer-frame simulation on AMD MI355X (gfx950).
 *
 * C ABI of libsframe.so.  The library simulates a quantum circuit of Clifford
 * gates, non-Clifford phase gates and Z-basis measurements on one stabilizer
 * frame (Garcia & Markov, "Simulation of Quantum Circuits via Stabilizer
 * Frames", Definition 1): a stabilizer matrix shared by a set of phase vectors,
 * each with a complex amplitude, such that the state is
 *   Psi = sum_j a_j psi(M, sigma_j).
 * The calls follow the paper's problem statement (section 2.1: initialise a
 * basis state, apply the gates one at a time, measure) and its frame
 * operations (section 3: ROTATE, COFACTOR; section 4: the gate rules and
 * "Measuring F").  Calls marked "not in the paper" are additions of this
 * library (batching, graphs, serving, tuning, profiling).
 *
 * Conventions
 *  - Qubit q of a packed bit vector is word q>>6, bit q&63; W = ceil(n/64).
 *  - Tableau rows are returned as W words of x bits followed by W words of z
 *    bits; literal (x,z) = 00 I, 01 Z, 10 X, 11 Y (section 2.2).  The returned
 *    tableau is the fully reduced row echelon form over the columns
 *    x_0..x_{n-1}, z_0..z_{n-1}, rows sorted by pivot (X-block first, as in
 *    Figure 2b); it carries no signs.
 *  - Phase vector bit i (1 = sign -1) belongs to row i of that tableau.
 *  - The amplitude a_j refers to psi(M, sigma_j) normalised with a real
 *    positive amplitude at the smallest basis string of its support, where
 *    qubit 0 is the most significant bit of a basis index.
 *  - Frame elements are returned in ascending order of sum_i sigma_i 2^i, with
 *    |a| > 1e-12 (smaller amplitudes are dropped after every merge).
 *  - A measurement of qubit q gives outcome 1 exactly when
 *    u = (splitmix64 output k of the stream seeded with `seed`) >> 11, * 2^-53
 *    is below p(1); k counts the measurements of the state from 0.
 *
 * Ownership and errors: every call returns an sf_status; no exception or abort
 * crosses the ABI.  The caller owns every host buffer it passes.  The library
 * owns device memory (allocated through the sf_allocator hook, or hipMalloc
 * when the hook is NULL) and frees it in the matching *_destroy.  Work is
 * queued on the context's HIP stream; calls that return host data
 * synchronise that stream.  A context must be used by one host thread at a
 * time.  sf_last_error returns the message of the last failed call.
 */
#ifndef SFRAME_H
#define SFRAME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SF_OK = 0,
  SF_E_INVALID = 1,   /* malformed argument or circuit */
  SF_E_OOM = 2,       /* device allocation failed */
  SF_E_DEVICE = 3,    /* HIP runtime error */
  SF_E_TOO_LARGE = 4, /* frame bound exceeds the limit or the memory budget */
  SF_E_STATE = 5,     /* call not valid in the current state */
  SF_E_BUFSIZE = 6,   /* output buffer too small; size returned */
  SF_E_CANCELLED = 7
} sf_status;

/* Gate codes.  theta = pi * theta_num / theta_den for SF_PHASE / SF_CPHASE /
 * SF_CPHASE_D. */
typedef enum {
  SF_H = 0, SF_S = 1, SF_SDG = 2, SF_X = 3, SF_Y = 4, SF_Z = 5,
  SF_CNOT = 6,    /* q0 control, q1 target */
  SF_CZ = 7,
  SF_T = 8, SF_TDG = 9,
  SF_PHASE = 10,  /* diag(1, e^{i theta}) on q0 */
  SF_CPHASE = 11, /* diag(1,1,1,e^{i theta}) on (q0,q1); expanded at load into
                     three phase gates and two CNOTs */
  SF_TOF = 12,    /* Toffoli (q0,q1 controls, q2 target); expanded at load into
                     the 7-T Clifford+T network */
  SF_MEASURE = 13, /* Z-basis measurement of q0 */
  SF_CPHASE_D = 14, /* diag(1,1,1,e^{i theta}) on (q0,q1), direct form (Eq. 3):
                       cofactor on q0 and q1, then the phase on the elements
                       where both read 1; theta a multiple of pi is I or CZ */
  SF_TOF_D = 15     /* Toffoli (q0,q1 controls, q2 target), direct form (Eq. 2):
                       cofactor on both controls, then X on q2 for the elements
                       where both read 1 */
} sf_op;

typedef struct {
  uint32_t op, q0, q1, q2;
  int64_t theta_num, theta_den;
} sf_gate;

/* Device allocator hook.  alloc returns device memory of `bytes` usable on
 * `stream` (NULL on failure); free releases it. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, size_t bytes, void* stream, void* user);
  void* user;
} sf_allocator;

typedef struct sf_ctx sf_ctx;
typedef struct sf_circuit sf_circuit;
typedef struct sf_state sf_state;
typedef struct sf_server sf_server;
typedef struct sf_graph sf_graph;

/* Not in the paper (runtime set-up).
 * Create a context on HIP device `device` that queues work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  `alloc` may be NULL.
 * hbm_budget_bytes bounds the device memory of all states (0 = no bound). */
sf_status sf_ctx_create(int device, void* hip_stream, const sf_allocator* alloc,
                        uint64_t hbm_budget_bytes, sf_ctx** out);
sf_status sf_ctx_destroy(sf_ctx* ctx);
const char* sf_last_error(const sf_ctx* ctx);

/* Section 2.1 (the circuit C as a gate sequence) and section 4 (the gate
 * rules: Eq. 2 Toffoli, Eq. 3 controlled phase, the T rule of the
 * technology-dependent decompositions); the frame bound follows COFACTOR
 * (section 3: a frame keeps or doubles its size).
 * Validate and load a circuit on n_qubits (1..2048).  Qubit indices must be
 * < n_qubits and distinct within a gate; theta_den != 0 for phase gates.
 * Loading rewrites phase gates whose angle is a multiple of pi/2 into
 * I/S/Z/S-dagger, expands SF_CPHASE and SF_TOF, and runs the tableau track
 * once to bound the frame: every frame of the run has at most 2^bound
 * elements (the dimension of the affine hull of its phase vectors).
 * Returns SF_E_TOO_LARGE when the bound exceeds 29.
 * Circuits on more than 256 qubits must be stabilizer circuits (Clifford
 * gates, phase gates at multiples of pi/2, measurements; the
 * random-stabilizer-circuit experiment of section 6), else SF_E_INVALID.
 * Their frames keep one element (bound 0) with the stabilizer rows in device
 * memory ("wide" states): they run through sf_step, sf_run, sf_measure and
 * sf_batch_run (one workgroup per frame), are reset by sf_state_reset and
 * read by the readout calls; sf_batch_run_noalloc, sf_batch_reset,
 * sf_batch_graph and sf_serve_submit refuse them with SF_E_INVALID. */
sf_status sf_circuit_load(sf_ctx* ctx, uint32_t n_qubits, const sf_gate* gates, size_t n_gates,
                          sf_circuit** out);
/* Not in the paper (admission).  Frame bound (log2) and the device bytes a
 * state of this circuit needs. */
sf_status sf_circuit_info(const sf_circuit* c, uint64_t* max_frame_bound_log2, uint64_t* projected_bytes);
sf_status sf_circuit_destroy(sf_circuit* c);

/* Section 2.1 (the simulation starts from a basis state) and Figure 2a
 * (the basis form of its stabilizer matrix: row q = Z_q, sign b_q).
 * Allocate a state and set it to the basis state |b>: basis_bits holds W
 * words, bit q = b_q (NULL = all zeros).  `seed` seeds the measurement coin. */
sf_status sf_state_init(sf_ctx* ctx, const sf_circuit* c, const uint64_t* basis_bits, uint64_t seed,
                        sf_state** out);
sf_status sf_state_destroy(sf_state* s);
/* As sf_state_init (section 2.1, Figure 2a), on an existing state.
 * Set an existing state back to |b> with a new seed, without allocating;
 * the circuit restarts from its first gate.  Asynchronous. */
sf_status sf_state_reset(sf_state* s, const uint64_t* basis_bits, uint64_t seed);
/* Not in the paper (a bound on |F| of Definition 1).
 * Dimension of the affine hull of the current phase vectors (|F| <= 2^d);
 * synchronises. */
sf_status sf_state_dim(sf_state* s, uint32_t* d);

/* Section 3 (ROTATE with global-phase maintenance, Eq. 1; COFACTOR) and
 * section 4 (non-Clifford gates, "Measuring F"): the gates applied one at a
 * time as in the problem statement of section 2.1.
 * Queue up to max_gates further gates of the circuit (counted as given to
 * sf_circuit_load); stops after each measurement.  *gates_applied receives
 * the number queued (0 at the end of the circuit).  Asynchronous. */
sf_status sf_step(sf_state* s, size_t max_gates, size_t* gates_applied);
/* As sf_step (sections 3 and 4), to the end of the circuit.
 * Queue every remaining gate.  Asynchronous. */
sf_status sf_run(sf_state* s);
/* Not in the paper (batching of independent frames; each frame follows
 * sections 3 and 4).
 * Run every remaining gate of n_states states (all of this context) as one
 * batch: per round, the tableau tracks of all frames share one launch (one
 * wavefront each) and the element kernels of all frames share one launch per
 * segment.  Results are identical to running each state alone.  When some
 * circuit has ranges that end without a measurement, the tracks of the next
 * round run on a second stream that the context keeps, beside the current
 * round's other kernels (the context's stream waits for that stream before
 * the call returns).  The per-round launch descriptors are staged through
 * pinned host memory that the context keeps (allocated on first use, freed
 * by sf_ctx_destroy).  Synchronises. */
sf_status sf_batch_run(sf_ctx* ctx, sf_state* const* states, size_t n_states);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not allocate, harnesses that forbid it).
 * sf_batch_run without any allocation: the per-round launch descriptors and
 * the error-gather table go to an 8 MiB device array of the library (one per
 * device, kept until the process ends) instead of memory from the allocator
 * hook, and the descriptors are copied from pageable host memory.  A frame of
 * more than 128 qubits whose per-gate record buffer does not exist yet runs
 * with the in-kernel phase evaluation instead of allocating it.  Results are
 * those of sf_batch_run.  SF_E_TOO_LARGE (nothing queued) when the states
 * would need more than 8 MiB of descriptors and gather table: about
 * n_states x (212 + 4 x (most segments of one range + 2)) bytes.  Calls on
 * one device share the array: calls that
 * overlap in time on one device (other host threads or streams) race and
 * must be serialised by the caller.  Synchronises. */
sf_status sf_batch_run_noalloc(sf_ctx* ctx, sf_state* const* states, size_t n_states);
/* Section 4, "Measuring F" (with COFACTOR of section 3).
 * Measure qubit q in the Z basis now, between circuit gates (the state must
 * be at a gate boundary, as after sf_step).  Same rule and random stream as
 * a MEASURE gate at this point of the circuit: the outcome takes the next measurement index, so later
 * circuit measurements draw the following ones.  *outcome receives 0 or 1.
 * Synchronises.  SF_E_INVALID for q >= n; SF_E_TOO_LARGE (state unchanged)
 * if after this measurement the rest of the circuit would need more frame
 * elements than the state was sized for. */
sf_status sf_measure(sf_state* s, uint32_t q, int* outcome);
/* Not in the paper (batching).
 * sf_state_reset for many states with one kernel launch: bases holds 4 words
 * per state (bit q of state i at bases[4 i + q / 64]; NULL: |0...0>), seeds
 * one per state (NULL: 0).  Synchronises. */
sf_status sf_batch_reset(sf_ctx* ctx, sf_state* const* states, size_t n_states, const uint64_t* bases,
                         const uint64_t* seeds);
/* Not in the paper (batching, recorded once as a HIP graph).
 * Graph form of sf_batch_run for frames that are run again and again.  Plans every round of a run of the given states
 * from their initial basis states and records the initialisation and all
 * launches as one hipGraph of kernel nodes; basis[i] (W words, or NULL for
 * |0...0>) and seeds[i] are the inputs of frame i (basis and seeds may be
 * NULL).  The states stay bound to the graph until sf_graph_destroy:
 * sf_state_destroy on them returns SF_E_STATE, and so does an sf_measure that
 * would have to grow their outcome buffers.  Synchronises. */
sf_status sf_batch_graph(sf_ctx* ctx, sf_state* const* states, size_t n_states, const uint64_t* const* basis,
                         const uint64_t* seeds, sf_graph** out);
/* Not in the paper.  Change the inputs of frame i for the next launch. */
sf_status sf_graph_set_input(sf_graph* g, size_t i, const uint64_t* basis_bits, uint64_t seed);
/* Not in the paper.
 * Re-initialise every frame of the graph from its inputs and run all its
 * gates (asynchronous, one graph launch on the context's stream).  Results
 * are those of sf_state_reset + sf_batch_run with the same inputs. */
sf_status sf_graph_launch(sf_graph* g);
/* Not in the paper.  Synchronises, frees the graph and releases its states. */
sf_status sf_graph_destroy(sf_graph* g);
/* Not in the paper (tuning).
 * Autotuner of the elementwise frame kernels (segment update and measurement
 * filter): for every hull
 * dimension d in [d_lo, d_hi] (0 <= d_lo <= d_hi <= 29) it times the segment
 * kernel over 2^d slots at each candidate shape (64/128/256 threads per
 * block x 1..32 slots per thread) and keeps the fastest for later launches of
 * this context.  Results do not depend on the shape.  blocks, grids and ms
 * (optional, d_hi - d_lo + 1 entries) receive the choice and its time per
 * launch.  Allocates 16 * 2^d_hi bytes of scratch while it runs.
 * Synchronises. */
sf_status sf_autotune(sf_ctx* ctx, int d_lo, int d_hi, int* blocks, int* grids, float* ms);
/* Not in the paper (tuning).
 * The context's launch tuning, so that a caller can keep it across
 * processes: the elementwise kernels' shape per hull dimension d
 * (SF_TUNE_DIMS entries, d = 0..30: threads per block and blocks) and the
 * number of phase-kernel wavefronts a batched launch aims for (each walks a
 * chunk of consecutive gates; default 65536).  sf_tuning_get copies it out
 * (any pointer may be NULL).  sf_tuning_set installs it: blocks and grids
 * both NULL keeps the shapes; a block other than 64, 128 or 256, a grid
 * outside 1..2^24 or phase_waves < 1 returns SF_E_INVALID and changes
 * nothing.  Results never depend on these values. */
#define SF_TUNE_DIMS 31
sf_status sf_tuning_get(const sf_ctx* ctx, int* blocks, int* grids, int* phase_waves);
sf_status sf_tuning_set(sf_ctx* ctx, const int* blocks, const int* grids, int phase_waves);
/* Not in the paper.  Wait for queued work; reports device-side failures of
 * the queued steps. */
sf_status sf_sync(sf_state* s);

/* Section 4, "Measuring F": the outcomes drawn so far.
 * Measurement outcomes so far (synchronises).  *count receives their number;
 * at most cap are written. */
sf_status sf_outcomes(sf_state* s, uint8_t* out, size_t cap, size_t* count);
/* Definition 1: the size |F| of the frame.
 * Number of frame elements |F| (synchronises). */
sf_status sf_frame_size(sf_state* s, uint64_t* K);
/* Definition 1 (the frame: stabilizer matrix M and the pairs of phase vector
 * sigma_j and amplitude a_j), with M in the echelon form of Invariant 1.
 * Read the frame in canonical form (synchronises): tableau (n rows of 2W
 * words), sigma (K rows of W words), amp (K interleaved re,im).  With
 * cap_K < K nothing is written, *K_out = K and SF_E_BUFSIZE is returned.
 * Any output pointer may be NULL. */
sf_status sf_read_frame(sf_state* s, uint64_t* tableau, uint64_t* sigma, double* amp, size_t cap_K,
                        size_t* K_out);
/* Not in the paper.
 * Gates of the circuit applied so far and whether a measurement result was
 * fragile (|u - p(1)| < 1e-12 or p(outcome) = 0). */
sf_status sf_state_info(sf_state* s, size_t* gates_done, int* fragile);

/* Not in the paper (serving with continuous batching; each job's frame
 * follows sections 3 and 4).  Queued jobs are considered in arrival order
 * and admitted while their projected device bytes (sf_circuit_info) fit
 * budget_bytes (0 = no bound) and fewer than max_resident jobs are resident;
 * a job that does not fit yet is passed by later jobs that do, in at most 16
 * ticks, after which nothing behind it is admitted before it.  A job whose
 * state cannot be allocated waits while others are resident and fails (status
 * 4) when none is; a resident job whose round cannot be planned (its buffers
 * cannot be allocated) fails and the other jobs go on.  Each sf_serve_tick
 * admits what fits, runs one batched round over all resident frames (each
 * advances to its next measurement or to its end, or, with tick_segments > 0,
 * stops earlier right after its tick_segments-th non-Clifford phase gate, so
 * that long measurement-free jobs yield to new arrivals), synchronises and
 * retires finished jobs, whose memory stays reserved until sf_serve_release.
 * A job's result does not depend on what else is resident or on
 * tick_segments.  Job status: 0 queued, 1 resident, 2 done, 3 cancelled,
 * 4 failed.  sf_serve_submit returns SF_E_TOO_LARGE for a job that can never
 * fit. */
sf_status sf_serve_create(sf_ctx* ctx, uint64_t budget_bytes, uint32_t max_resident, uint32_t tick_segments,
                          sf_server** out);
sf_status sf_serve_submit(sf_server* sv, const sf_circuit* c, const uint64_t* basis_bits, uint64_t seed,
                          uint64_t* job_id);
sf_status sf_serve_tick(sf_server* sv, uint32_t* n_resident, uint32_t* n_queued);
/* Not in the paper.  *state receives the finished state (owned by the
 * server) when status is 2. */
sf_status sf_serve_poll(sf_server* sv, uint64_t job_id, int* status, sf_state** state);
sf_status sf_serve_release(sf_server* sv, uint64_t job_id);
sf_status sf_serve_cancel(sf_server* sv, uint64_t job_id);
sf_status sf_serve_stats(sf_server* sv, uint64_t* ticks, uint64_t* admitted, uint64_t* rejected,
                         uint64_t* used_bytes);
sf_status sf_serve_destroy(sf_server* sv);

/* Not in the paper (profiling).
 * Per-kernel device time, measured with HIP events on the context stream.
 * sf_profile(ctx, mask) starts collecting (and clears the totals) for the
 * kernel kinds whose bit is set in mask (-1: all), 0 stops.
 * sf_profile_read returns total milliseconds and launch counts per kernel
 * kind: 0 tableau track, 1 segment (phase + cofactor; for frames of at most
 * 256 slots the whole element stage of a round), 2 measurement reduction,
 * 3 unused (the coin is drawn by the filter kernel; kept for the numbering),
 * 4 measurement coin and filter, 5 readout, 6 state initialisation, 7
 * per-gate phase evaluation and 8 per-segment phase fit (the parallel part of
 * the tableau track of frames of up to 128 qubits).  Both synchronise. */
sf_status sf_profile(sf_ctx* ctx, int enable);
sf_status sf_profile_read(sf_ctx* ctx, double* ms, uint64_t* launches, int n_kinds);
/* Not in the paper (profiling).
 * Shader clocks the tableau track of this state spent per phase since the
 * last init/reset: 0 saving the pre-gate tableau, 1 column updates, 2 echelon
 * repair, 3 index and b* images, 4 phase sampling, 5 fitting of Hadamard
 * terms, 6 cofactor/measurement steps, 7 total, 8-10 parts of the repair (checks,
 * row products, replay on the hull), 11 spare.  Synchronises. */
sf_status sf_state_cycles(sf_state* s, uint64_t* cycles, int n);

#ifdef __cplusplus
}
#endif
#endif /* SFRAME_H */
