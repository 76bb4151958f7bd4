/*
 * pauliprop -- Heisenberg-picture Pauli propagation on MI355X (gfx950).
 *
 * Computes <O>(theta) = <0...0| U(theta)^dag O U(theta) |0...0> for a
 * parameterized circuit U = g_m ... g_1 (Sec. I: a PQC of m fixed and
 * parameterized gates) by propagating the observable O, a real-weighted sum
 * of n-qubit Pauli strings (Sec. II-A), backwards through the gates:
 *   - a Clifford gate (H, S, CX) maps every string to one string with a sign
 *     (Sec. II-A: constant-time local update; CX list of Sec. III-C;
 *     H and S rows of Table I, applied as the inverse map g^dag P g);
 *   - a rotation R_sigma(theta) = exp(-i theta sigma/2) keeps every string that
 *     commutes with sigma and splits every anticommuting one into a cos(theta)
 *     string and a sin(theta) string (R rows of Table I, Example 1);
 *   - strings that coincide are merged by summing their weights, with no
 *     pruning (Sec. III-B expand/reduce, eq. (7), Examples 3 and 4);
 *   - <O> is the sum of the weights of the strings made of I and Z only.
 *
 * Conventions used by every entry point:
 *   qubit q is bit q of the x and z words; I=(0,0) X=(1,0) Y=(1,1) Z=(0,1);
 *   Y is the Hermitian Pauli; weights are real; gates are given in
 *   application order g_1 ... g_m; rotations read their angle from
 *   theta[param[g]].
 *
 * Errors: every function returns a pp_status; on failure pp_last_error()
 * returns a thread-local message and the object is left as it was.
 * Asynchrony: functions taking a stream enqueue work on that HIP stream
 * (a hipStream_t passed as void*, NULL = the null stream) and return; device
 * outputs are valid once the stream has reached that point.  Functions that
 * return host data synchronize: pp_get_terms its stream, pp_get_stats the
 * device.  A circuit keeps no stream handle of a past call.
 * Threading: one circuit must not be used by two threads at once; distinct
 * circuits are independent.
 */
#ifndef PAULIPROP_H
#define PAULIPROP_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define PP_API __attribute__((visibility("default")))
#else
#define PP_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pp_status {
    PP_OK = 0,
    PP_ERR_INVALID = 1,  /* bad argument: the object is unchanged */
    PP_ERR_NOMEM = 2,    /* device or host allocation failed */
    PP_ERR_DEVICE = 3,   /* a HIP call failed (message kept) */
    PP_ERR_CAPACITY = 4, /* the term set does not fit the configured capacity */
    PP_ERR_STATE = 5,    /* call order: gates / theta / observable missing */
    PP_ERR_BUSY = 6      /* server: no slot or memory free yet */
} pp_status;

/* Gate codes (Sec. III-A: an instructor is {gate, wire, theta}). */
typedef enum pp_op { PP_H = 0, PP_S = 1, PP_CX = 2, PP_RX = 3, PP_RY = 4, PP_RZ = 5 } pp_op;

/* Storage type of the weights.  Arithmetic inside a pass is FP64 in both. */
typedef enum pp_dtype { PP_F64 = 0, PP_F32 = 1 } pp_dtype;

/* Engine.
 *  DENSE : direct addressing; the weight of string P lives at slot
 *          index(P) of a 4^n array (the paper's lambda vector indexed
 *          0 ... 4^n - 1, Sec. III-B), so merging duplicates is implicit.
 *          Practical for n <= 13.
 *  SPARSE: an explicit list of weighted strings.  Exact runs with n <= 31
 *          propagate in the Clifford frame: Clifford gates are folded on the
 *          host into the axis of the next rotation (a multi-qubit Pauli),
 *          so the stored strings never move and a rotation splits them in
 *          one kernel, pairing duplicates through a hash index.  Otherwise
 *          each pass applies a run of Clifford gates and one rotation,
 *          appends the split strings by wave-ballot compaction, then merges
 *          duplicates with a radix sort and a segmented FP64 sum.
 *          n <= 64; the capacity is set with PP_OPT_MAX_TERMS.
 *  AUTO  : DENSE when 4^n slots fit the memory budget, else SPARSE. */
typedef enum pp_engine { PP_ENGINE_AUTO = 0, PP_ENGINE_DENSE = 1, PP_ENGINE_SPARSE = 2 } pp_engine;

/* Per-circuit options (pp_circuit_set_option). */
typedef enum pp_option {
    PP_OPT_TRACK_TERMS = 0, /* 1: keep the exact string set and count term
                               updates (needed by pp_get_terms in DENSE);
                               0 (default): weights only, fastest */
    PP_OPT_TILE_QUBITS = 1, /* DENSE, n >= 8: qubits per LDS tile (4..7);
                               0 = autotuned default */
    PP_OPT_MAX_TERMS = 2,   /* SPARSE: capacity of the term list (default
                               min(4^n, 2^24), at most 2^29); the buffers
                               hold 2x this */
    PP_OPT_USE_GRAPH = 3,   /* 1: replay a captured hipGraph for pp_evaluate
                               (tiled DENSE, and SPARSE: its whole pass and
                               merge sequence, which needs no host sync), for
                               pp_gradient (the whole Heisenberg + adjoint
                               sweep, a training step's launch sequence) and
                               for pp_evaluate_batch when every circuit of the
                               batch sets it (the whole step: start weights,
                               maps, LDS-resident circuits, every tile pass
                               and the readouts, captured once per set of
                               circuits and output array); theta is read
                               from device memory at replay */
    PP_OPT_BLOCK = 4,       /* threads per workgroup (64..1024), 0 = default */
    PP_OPT_SPARSE_FRAME = 5, /* SPARSE, exact runs with n <= 31: 1 (default)
                               propagates in the Clifford frame (Clifford
                               gates folded into the rotation axes on the
                               host, one kernel per rotation, duplicates
                               found through a hash index); 0 uses the
                               sort-merge pass of every rotation.  Same
                               strings and weights; truncated runs and
                               n > 31 always use sort-merge */
    PP_OPT_FRAME_RAMP = 6   /* DENSE without term tracking: t in 1..24 starts
                               the Heisenberg sweep in the Clifford frame,
                               where the set holds only its strings (it grows
                               from the observable's toward 4^n, Sec. II-B),
                               and hands the strings to the 4^n array once
                               the set could exceed 4^n / 2^t: the frame
                               takes the longest suffix of gates over which
                               (observable terms) x 2^(rotations) stays
                               within that limit, which is also the frame's
                               capacity.  0 (default) is the 4^n array from
                               the first gate.  Results agree within
                               rounding (the merge order differs).  Such a
                               circuit is evaluated one by one inside
                               pp_evaluate_batch and served through the
                               general path; pp_evaluate_thetas and
                               pp_evaluate_noalloc refuse it (PP_ERR_STATE) */
} pp_option;

typedef struct pp_circuit pp_circuit;

typedef struct pp_stats {
    int64_t term_updates; /* U = sum over gates of the set size entering the
                             gate, from the last tracked (or SPARSE) run */
    int64_t final_terms;  /* strings in the final set (tracked or SPARSE) */
    int64_t gates;        /* m */
    int64_t ops;          /* device operations after fusion */
    int64_t passes;       /* passes over the term set per evaluation */
    int64_t launches;     /* kernel launches per evaluation */
    int64_t bytes_per_eval; /* algorithmic HBM bytes of one evaluation */
    int32_t engine;       /* pp_engine actually used */
    int32_t tile_qubits;  /* DENSE: qubits per tile (n if LDS-resident) */
    int32_t overflow;     /* SPARSE: 1 if the capacity was exceeded */
    int32_t reserved;
} pp_stats;

/* Accumulated device time of one kernel class (pp_profile_read). */
typedef struct pp_kernel_time {
    char name[32];      /* "tile_pass", "resident", "compose", "dense_init",
                           "readout", "sparse_pass", "sparse_merge" */
    int64_t launches;   /* launches timed since profiling was enabled */
    double total_ms;    /* sum of event-measured durations */
} pp_kernel_time;

/* ------------------------------------------------------- device memory */
/* Where the library's device buffers come from (the per-circuit weights,
 * schedules and scratch, the server's pool).  alloc(bytes, stream, user)
 * returns device memory of at least `bytes` bytes usable on any stream once
 * it returns, or NULL on failure (the calling entry point then returns
 * PP_ERR_NOMEM and leaves its object usable: a later call with memory
 * available succeeds); `stream` is the stream of the first use or NULL.
 * free(ptr, bytes, stream, user) takes back a block of this allocator; the
 * library synchronizes the device first, so no enqueued work still uses it.
 * Both may be called from the library's own threads (the serving loop and
 * its preparation threads). */
typedef struct pp_allocator {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, size_t bytes, void *stream, void *user);
    void *user;
} pp_allocator;

/* Installs the allocator for every later device allocation (a copy of *a is
 * kept); NULL restores the default, the stream-ordered pool (hipMallocAsync
 * on an internal stream, synchronized before the buffer is handed out).  A
 * block is always returned to the allocator that made it.  The Python
 * binding installs torch's caching allocator.  PP_ERR_INVALID if alloc or
 * free is NULL.  This is the instructor/gate boundary of Sec. III-A with the
 * device memory owned by the framework above it. */
PP_API pp_status pp_set_allocator(const pp_allocator *a);

/* Bytes and blocks of device memory the library holds right now (all
 * circuits, servers and scratch of the process). */
PP_API pp_status pp_memory_in_use(int64_t *bytes, int64_t *blocks);

/* Library version string; never NULL. */
PP_API const char *pp_version(void);

/* Message of the last failure on the calling thread ("" if none). */
PP_API const char *pp_last_error(void);

/* Creates an empty circuit on the current HIP device: n qubits starting in
 * |0...0> (Sec. II-A: the initial state is stabilized by the Z_j).  n_qubits
 * in [1, 64] (DENSE additionally needs 4^n slots in memory).  *out receives
 * the handle; release it with pp_circuit_destroy.  No device memory is
 * allocated yet. */
PP_API pp_status pp_circuit_create(int32_t n_qubits, pp_dtype dtype, pp_engine engine, pp_circuit **out);

/* Releases the circuit and every device buffer it owns.  NULL-safe.  The
 * caller must make sure no enqueued work still uses it. */
PP_API void pp_circuit_destroy(pp_circuit *c);

/* Loads the gate list (host arrays of length m, copied during the call):
 * the instructors {gate, wire, theta} of Sec. III-A in application order.
 * A device array for the angles is allocated (PP_ERR_NOMEM on failure, the
 * circuit keeping its previous gates).
 * op[g] is a pp_op; q0[g] the qubit (CX control); q1[g] the CX target, else
 * ignored; param[g] in [0, n_params) for rotations, ignored otherwise.
 * Errors: PP_ERR_INVALID for an unknown op, a qubit outside [0, n),
 * CX with q0 == q1 or a parameter index outside [0, n_params). */
PP_API pp_status pp_circuit_load_gates(pp_circuit *c, int64_t m, const uint8_t *op, const int32_t *q0,
                                const int32_t *q1, const int32_t *param, int32_t n_params);

/* Sets the n_params angles of the parameterized gates (the theta of the
 * PQC, Sec. I).  on_device = 0: theta is a host array (copied
 * before return); 1: theta is a device array read by the next evaluations
 * on `stream` (it must stay valid until they ran).  Non-finite angles are
 * not checked; they propagate NaN. */
PP_API pp_status pp_circuit_set_theta(pp_circuit *c, const double *theta, int32_t on_device, void *stream);

/* Sets the observable O = sum_k coeff[k] P(x[k], z[k]) (host arrays, copied):
 * a real-weighted sum of Pauli strings, the form every propagated operator
 * keeps (Sec. II-A, the lambda_j P_j of the generator expansion).  Bits at
 * or above n must be zero (PP_ERR_INVALID).  Repeated strings are summed. */
PP_API pp_status pp_circuit_set_observable(pp_circuit *c, int64_t n_terms, const uint64_t *x,
                                    const uint64_t *z, const double *coeff);

/* Sets a pp_option; takes effect at the next evaluation.  PP_ERR_INVALID
 * for an unknown key or a value out of range (the circuit unchanged). */
PP_API pp_status pp_circuit_set_option(pp_circuit *c, pp_option key, int64_t value);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * evaluation as pp_evaluate for a DENSE circuit without term tracking, with
 * the same result bit for bit, but every working buffer (the 4^n weights,
 * the composed per-wire maps, the launch descriptors) in a static device
 * array of the library, 24 MiB per device, held until the process ends.
 * The call allocates nothing and copies nothing from the host: it enqueues
 * kernel launches on `stream` only.  It reads the circuit's schedule from the
 * device, so the circuit must have been evaluated once with pp_evaluate (or
 * pp_evaluate_batch, or served) since its gates, observable or options last
 * changed: PP_ERR_STATE otherwise, and for SPARSE or tracked circuits.
 * PP_ERR_CAPACITY when the working set does not fit the array (4^n weights
 * plus 72 bytes per map plus 80 bytes per pass: n <= 10 in FP64, n <= 11 in
 * FP32).  The circuit's own weights are left as they were.  Every call on
 * one device shares that device's array, which keeps the last call's
 * contents (each call rewrites all it reads): calls that overlap on one
 * device race, so enqueue them on one stream or serialize them. */
PP_API pp_status pp_evaluate_noalloc(pp_circuit *c, void *stream, double *d_expval);

/* Enqueues one evaluation of <O> = <0...0| U^dag O U |0...0> (measurement
 * of Sec. II-A from the propagated strings: only strings of I and Z have a
 * nonzero expectation in |0...0>); d_expval is caller-owned device memory
 * for one double.  PP_ERR_STATE if gates, theta or the observable are
 * missing; PP_ERR_NOMEM if the first evaluation's buffers cannot be
 * allocated (the circuit stays usable). */
PP_API pp_status pp_evaluate(pp_circuit *c, void *stream, double *d_expval);

/* Evaluates `count` independent circuits in batched launches on `stream`
 * (the independent units of Sec. IV run side by side; the PSR of Sec. I
 * needs 2m evaluations per gradient): circuits that fit one workgroup's LDS
 * run one per workgroup in a single launch per size class, larger ones share
 * multi-circuit tiled passes.  d_expvals: caller-owned device array of
 * `count` doubles, in input order.  Each circuit's result is bit-identical
 * to its own pp_evaluate.  PP_ERR_INVALID if a circuit appears twice (the
 * launches would update its one weight array from two places).  When every
 * circuit sets PP_OPT_USE_GRAPH (and all are untracked DENSE), the step is
 * captured as one hipGraph the first time this set of circuits meets this
 * output array, and replayed afterwards (same results bit for bit); the
 * capture is dropped when the set, a schedule or the array changes. */
PP_API pp_status pp_evaluate_batch(pp_circuit *const *cs, int64_t count, void *stream, double *d_expvals);

/* Parameter sweep (the 2m parameter-shift evaluations of Sec. I, a scan
 * over theta): enqueues <O> of circuit c at `count` parameter vectors.
 * thetas: count x n_params doubles, row-major, host memory (on_device = 0,
 * copied before return) or device memory (on_device = 1, read on `stream`).
 * d_expvals: caller-owned device array of `count` doubles.  All sets share
 * the schedule: each tile pass of all of them is one launch (LDS-resident
 * circuits: one launch), with per-set maps and 4^n weights that the circuit
 * keeps between calls (count x 4^n x sizeof(weight) bytes of device memory;
 * PP_ERR_NOMEM when that does not fit).  Each result is bit-identical to
 * pp_evaluate with the same theta.  DENSE engine without term tracking only
 * (else PP_ERR_STATE); theta set with pp_circuit_set_theta is not used. */
PP_API pp_status pp_evaluate_thetas(pp_circuit *c, int64_t count, const double *thetas, int32_t on_device,
                                    void *stream, double *d_expvals);

/* Enqueues <O> and its gradient with respect to theta (adjoint method on the
 * DENSE engine): d_expval one double, d_grad n_params doubles (caller-owned
 * device memory; contributions of gates sharing a parameter are summed).
 * The gradient the parameter-shift rule of Sec. I gives with 2m evaluations
 * comes from two sweeps: the observable's weights c_k (Heisenberg picture)
 * and the state's Pauli coefficients r_k (the density operator as a sum over
 * Pauli strings, eqs. (2)-(3)) are joined at every rotation,
 * d<O>/d theta_k = c_k^T A_sigma r_k.  checkpoint_every_gates > 0 stores
 * the propagated set every that many gates and recomputes inside each
 * segment; 0 picks a default.  FP64 only. */
PP_API pp_status pp_gradient(pp_circuit *c, void *stream, int32_t checkpoint_every_gates, double *d_expval,
                      double *d_grad);

/* Parameter-shift gradient (Sec. I: each rotation's derivative is half the
 * difference of two evaluations at its angle +- pi/2, exact for generators
 * with eigenvalues +-1/2): enqueues the 2R shifted evaluations of the R
 * rotation gates as one parameter sweep (pp_evaluate_thetas) of a private
 * copy of the circuit in which every rotation has a parameter of its own,
 * and sums the halved differences per parameter in gate order, all on the
 * device.  d_grad: caller-owned device array of n_params doubles.  The
 * private copy, its 2R x R shifted sets and its sweep buffers (2R x 4^n
 * weights for tiled circuits) stay allocated with c.  DENSE engine without
 * term tracking (else PP_ERR_STATE); PP_ERR_CAPACITY when 2R^2 exceeds
 * 2^27 doubles. */
PP_API pp_status pp_psr_gradient(pp_circuit *c, void *stream, double *d_grad);

/* Density matrix rho = U(theta) |0...0><0...0| U(theta)^dag (the paper's toDM
 * task; density operator as a sum over the stabilizer group, eq. (3), decoded
 * as in Sec. III-D).  The 2^n group strings Z^z are propagated through the
 * circuit in the Schrodinger picture on the DENSE engine (an internal circuit
 * of the inverse gates, built on the first call after pp_circuit_load_gates;
 * its 4^n weights stay allocated with c), then a Walsh-Hadamard transform per
 * X part turns the Pauli weights into matrix entries.  d_rho: caller-owned
 * device memory of 2 * 4^n doubles, row-major complex (real, imaginary)
 * pairs, rho[a][b] at 2 * (a * 2^n + b); bit q of a basis index is qubit q.
 * Uses the gates and theta of c (not its observable); the weight type follows
 * c's dtype, the decode is FP64.  n <= 12 (PP_ERR_INVALID above), PP_ERR_STATE
 * without gates or theta.  Enqueued on `stream`. */
PP_API pp_status pp_density_matrix(pp_circuit *c, void *stream, double *d_rho);

/* Truncated propagation (approximate; not part of the paper's exact method,
 * which keeps every string): SPARSE engine only (PP_ERR_STATE otherwise).
 * From the next evaluation on, a split child with more than max_weight
 * non-identity letters is not created, and after every merge a string with
 * more letters or with |weight| < min_abs_coeff is dropped.  Each dropped
 * string P of weight w changes <O> by at most |w| (|<psi|P|psi>| <= 1), so
 * the summed absolute dropped weight (pp_get_truncation) bounds the error.
 * min_abs_coeff = 0 and max_weight >= n (the defaults: 0, 64) is the exact
 * method.  PP_ERR_INVALID for min_abs_coeff < 0 or max_weight outside
 * [1, 64]. */
PP_API pp_status pp_circuit_set_truncation(pp_circuit *c, double min_abs_coeff, int32_t max_weight);

/* Summed absolute weight dropped by truncation during the last SPARSE
 * evaluation (0 for an exact run); synchronizes `stream`.  PP_ERR_STATE
 * before a SPARSE evaluation. */
PP_API pp_status pp_get_truncation(pp_circuit *c, void *stream, double *dropped_abs);

/* Copies the final string set of the last evaluation to host arrays in
 * canonical order (by z, then x), synchronizing `stream`: the reduced
 * weighted string set of Sec. III-B (Examples 3 and 4).  DENSE with
 * PP_OPT_TRACK_TERMS = 1 for that evaluation returns the structural set (exact
 * zero weights included, as the paper's expand/reduce keeps them); without it,
 * the strings whose final weight is nonzero (tiled circuits only: an untracked
 * LDS-resident evaluation, n <= 7, keeps its weights on chip and gives
 * PP_ERR_STATE).  At most `capacity` strings are
 * written; *n_out receives the full count (PP_ERR_CAPACITY if larger). */
PP_API pp_status pp_get_terms(pp_circuit *c, void *stream, int64_t capacity, uint64_t *x, uint64_t *z,
                       double *coeff, int64_t *n_out);

/* Fills *out with the statistics of the last evaluation (synchronizes the
 * device; the evaluation's stream may no longer exist): the work of the Map stage of Sec. IV-B as term
 * updates, passes and algorithmic bytes. */
PP_API pp_status pp_get_stats(pp_circuit *c, pp_stats *out);

/* ----------------------------------------------------------- serving */
typedef struct pp_server pp_server;

/* Serving (no counterpart in the paper, whose PQC training loop of Sec. I
 * evaluates many independent circuits: here they arrive one by one).
 *
 * Starts a serving loop on its own host thread and HIP streams of the
 * current device, with four preparation threads that build and upload each
 * request's schedule as it is submitted.  Prepared requests are admitted in
 * submission order while at most max_active are in flight and the sum of
 * their footprints (4^n weights for tiled DENSE requests, the term capacity
 * for SPARSE or tracked ones, none for LDS-resident ones) stays within
 * mem_budget_bytes.  Tiled DENSE requests run in weight buffers of the
 * server's pool, returned at completion and reused; the pool (buffers in
 * use and free) never exceeds mem_budget_bytes, so the budget bounds the
 * device memory of the served weights.  Admitted requests share work: every
 * loop iteration issues one batched tile pass per (tile size, weight type)
 * holding the next pass of every active tiled request (requests join and
 * leave between iterations), while circuits that fit one workgroup's LDS run
 * whole beside the passes: the pending ones are launched together (one
 * workgroup each) on whichever of three side streams is idle.  Each
 * request's result is bit-identical to its own pp_evaluate.  Device buffers
 * come from the allocator of pp_set_allocator. */
PP_API pp_status pp_server_create(int64_t mem_budget_bytes, int32_t max_active, pp_server **out);

/* Bounds the requests submitted and not yet admitted: with max_queued > 0
 * pp_server_submit returns PP_ERR_BUSY (nothing queued) while that many
 * wait; 0 (the default) queues without bound. */
PP_API pp_status pp_server_set_queue_limit(pp_server *s, int64_t max_queued);

/* Queues an evaluation of circuit c (gates, theta and observable set) and
 * returns its ticket.  The server owns c until the request is done: the
 * caller must not use, change or destroy it before pp_server_poll reports
 * done.  The work is ordered after c's last pp_circuit_set_theta upload on
 * whatever stream it was made.  A served tiled DENSE circuit keeps no final
 * weights (pp_get_terms then gives PP_ERR_STATE).  Errors: PP_ERR_CAPACITY
 * if c alone exceeds the memory budget; PP_ERR_INVALID if c was submitted
 * and is not done yet; PP_ERR_BUSY if the queue limit is reached;
 * PP_ERR_STATE after pp_server_destroy has begun.  Planning errors are
 * reported by pp_server_poll. */
PP_API pp_status pp_server_submit(pp_server *s, pp_circuit *c, int64_t *ticket);

/* Non-blocking status of a ticket: *done = 1 once the result is on the
 * host; then *expval is <O> and *latency_us the time from submission to
 * completion seen by the serving thread.  A failed request reports done with
 * its pp_status returned.  PP_ERR_INVALID for an unknown ticket. */
PP_API pp_status pp_server_poll(pp_server *s, int64_t ticket, int32_t *done, double *expval, double *latency_us);

/* Blocks until every submitted request is done. */
PP_API pp_status pp_server_drain(pp_server *s);

/* Loop iterations and batched tile launches issued so far, and the largest
 * number of requests in flight at once. */
PP_API pp_status pp_server_counters(pp_server *s, int64_t *iterations, int64_t *tile_launches, int64_t *max_in_flight);

/* Bytes the weight pool holds now (buffers in use and free) and at most so
 * far; both stay within the memory budget. */
PP_API pp_status pp_server_pool_bytes(pp_server *s, int64_t *held, int64_t *peak);

/* Finishes the queued requests, stops the loop and releases the server and
 * its pool.  NULL-safe. */
PP_API void pp_server_destroy(pp_server *s);

/* ------------------------------------------------------------ tuning */
/* Library-wide tuning knobs (no counterpart in the paper; the shapes of the
 * Map-stage kernels of Sec. IV-B; set by the autotuner, read when a schedule is
 * built or a kernel launched):
 *   PP_TUNE_TILE_QUBITS: index = n (8..16), value = default tile qubits k
 *                        (4..7) for circuits without PP_OPT_TILE_QUBITS;
 *   PP_TUNE_TILE_KERNEL: index = k (4..7), value = 0 one 256-thread
 *                        workgroup per tile (512 for k = 7), 1 persistent
 *                        workgroups (256 threads; 512 for k = 7) that
 *                        prefetch the next tile, 2 (k <= 6) one
 *                        single-wave (64-thread) workgroup per tile, 3
 *                        (k = 6 only) one wave per tile holding the tile
 *                        in registers, LDS used only to change which three
 *                        qubits sit in registers, 4 (k = 6 only) the same,
 *                        persistent, prefetching the next tile.  Variants
 *                        1, 3 and 4 serve launches whose circuits have
 *                        n <= 14 (32-bit buffer offsets); larger ones run
 *                        variant 0.  Choosing 3 or 4 for k = 6, or leaving
 *                        them, re-plans a circuit at its next evaluation:
 *                        their schedules order each pass into register
 *                        segments.
 *   PP_TUNE_RESIDENT_BLOCK: index = n (5..7), value = 256, 512 or 1024
 *                        threads for the LDS-resident kernel (untracked runs).
 *   PP_TUNE_SORT_SHAPE: index = capacity class of a SPARSE circuit's term
 *                        buffers (0: up to 2^17 terms, 1: up to 2^21, 2:
 *                        larger), value = shape of the radix sort that
 *                        merges equal strings (reduce(), eq. (7)): 0 = 8 key
 *                        bits per pass, 8 terms per thread (256 threads);
 *                        1 = 8 bits, 4 terms; 2 = 8 bits, 16 terms; 3 = 7
 *                        bits, 8 terms (128 threads); 4 = 7 bits, 16 terms;
 *                        5 = 6 bits, 16 terms (64 threads).  Every shape is
 *                        a stable sort on the same key: same order, same
 *                        results.
 * The knobs are process-wide and not synchronized: set them while no
 * evaluation, batch or server is running (a server's requests are planned
 * on its preparation threads and launched later).
 * Variants 0, 1 and 2 give bit-identical results for a given tile size, and
 * so do 3 and 4; the two groups' schedules order commuting ops differently
 * and agree up to rounding.  k changes how ops are packed and therefore the
 * rounding, so a circuit keeps the k of its schedule.  The resident block size changes the order of the
 * final readout sum only. */
typedef enum pp_tune_key {
    PP_TUNE_TILE_QUBITS = 0,
    PP_TUNE_TILE_KERNEL = 1,
    PP_TUNE_RESIDENT_BLOCK = 2,
    PP_TUNE_SORT_SHAPE = 3
} pp_tune_key;
PP_API pp_status pp_tune_set(pp_tune_key key, int32_t index, int32_t value);
PP_API pp_status pp_tune_get(pp_tune_key key, int32_t index, int32_t *value);

/* Host-only planning introspection (no device needed): runs the DENSE
 * scheduler (the grouping of gates into operators of Sec. III-A, here tile
 * passes and per-wire maps, fed to the Map stage of Sec. IV-B) on a gate list and reports the number of device ops and passes
 * for tiles of k qubits (k = n: one LDS-resident pass).  compose = fold a
 * wire's single-qubit gates into one op; reorder = let gates on disjoint
 * qubits move past each other.  pass_ops (optional, capacity max_passes)
 * receives the op count of each pass.  Same validation as
 * pp_circuit_load_gates. */
PP_API pp_status pp_plan_dense_info(int32_t n_qubits, int64_t m, const uint8_t *op, const int32_t *q0,
                                    const int32_t *q1, const int32_t *param, int32_t n_params, int32_t k,
                                    int32_t compose, int32_t reorder, int64_t *n_ops, int64_t *n_passes,
                                    int32_t *pass_ops, int64_t max_passes);

/* Host-only introspection of the Clifford frame of a SPARSE schedule (no
 * device needed; n in [1, 31]): the sparse passes (in Heisenberg order, each
 * a run of Clifford gates closed by a rotation, or the trailing Clifford
 * gates) and for each the axis of its rotation in the stored frame, P = D
 * sigma D^dag with D the Clifford gates processed so far (Table I's
 * rotation rows conjugated by D): pmask[i] = its Pauli string packed as
 * (z << n) | x, sign[i] = +-1 with P = sign * that Hermitian Pauli,
 * rot_param[i] (-1 for the trailing Clifford gates), ngates[i]; xrows (n
 * entries, optional): bit j of the x part of a stored string's actual form
 * after every Clifford is the parity of its packed key masked by xrows[j].
 * Arrays of capacity max_passes; *n_passes receives the count.  Same
 * validation as pp_circuit_load_gates. */
PP_API pp_status pp_plan_sparse_frame(int32_t n_qubits, int64_t m, const uint8_t *op, const int32_t *q0,
                                      const int32_t *q1, const int32_t *param, int32_t n_params, int64_t max_passes,
                                      uint64_t *pmask, int32_t *sign, int32_t *rot_param, int32_t *ngates,
                                      uint64_t *xrows, int64_t *n_passes);

/* Kernel timing for measurement (the stage timings of Sec. V, taken with
 * HIP events): while enabled (on = 1), the library's
 * kernel launches are timed with HIP events recorded on the stream they are
 * launched on.  A run of consecutive tile passes (one call's passes on one
 * stream) is bracketed by one pair of events and each of its launches is
 * credited with the run's mean duration, so the passes still run back to
 * back; every other launch is bracketed by its own pair (each recorded event
 * delays the next kernel by a few microseconds).  The events carry no
 * system-scope fence.  on = 0 stops recording.  Not thread-safe; meant for
 * benchmarks. */
PP_API pp_status pp_profile_enable(int32_t on);

/* Synchronizes on the recorded events and writes up to `max` per-class
 * totals (launches and summed milliseconds) into out[], *n_out = classes
 * written; then clears the record. */
PP_API pp_status pp_profile_read(pp_kernel_time *out, int32_t max, int32_t *n_out);

#ifdef __cplusplus
}
#endif

#endif /* PAULIPROP_H */
