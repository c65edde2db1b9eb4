/*
 * qs.h -- C ABI of the full-amplitude state-vector library (libqs.so).
 *
 * Method: the full-amplitude ("Schrodinger") mode of Wang et al., "A quantum
 * circuit simulator and its applications on Sunway TaihuLight supercomputer"
 * (arXiv:2008.07140), Sec. 2.2 and Sec. 2.4, with the instruction set of
 * App. A-1.  The library keeps all 2^n complex amplitudes of an n-qubit state
 * in the device memory of one AMD Instinct MI355X (gfx950) and updates them in
 * place with hand-written HIP kernels.
 *
 * Conventions shared by every call
 *  - Qubit k is bit k of the amplitude index: i = sum_k i_k 2^k (Sec. 2.2,
 *    Eq. 1).  Amplitudes are stored interleaved (re, im) in index order:
 *    QS_C128 = two doubles per amplitude (16 B), QS_C64 = two floats (8 B).
 *  - A gate matrix on nt targets is 2^nt x 2^nt, row-major, given as (re, im)
 *    double pairs (2 * 4^nt doubles).  Bit (nt-1-b) of its row/column index is
 *    the value of targets[b]: targets[0] is the most significant bit, as in the
 *    CNOT / CR / TOFFOLI matrices of App. A-1 where the first listed qubit is
 *    the high bit.
 *  - Controls are |1>-controls (Eq. 3; App. A-1 CNOT/CZ/CR/TOFFOLI/CONTROL):
 *    the gate acts on the amplitudes whose control bits are all 1 and leaves
 *    the others unchanged.
 *  - Ownership: every host array passed in is owned by the caller and is only
 *    read (or written, for outputs) during the call; the library copies what
 *    it keeps.  Device memory is owned by the state unless it was borrowed
 *    with qs_create_from_buffer.
 *  - Ordering: calls that change a state are enqueued on the state's HIP
 *    stream and return before the device has finished.  Calls that return
 *    host data (qs_amplitudes, qs_probabilities, qs_norm, qs_apply_noisy_gate,
 *    qs_run_circuit with noise sites, qs_profile_query) synchronise the stream.
 *  - Errors: every call returns a qs_status and never aborts.  Arguments are
 *    validated on the host before anything is enqueued, so a call that fails
 *    validation leaves the state unchanged.  qs_last_error() returns a text
 *    description of the last failure on the calling thread (the counterpart
 *    of the error log of App. A-2).
 *  - Sizes: 1 <= n <= QS_MAX_QUBITS; a gate has 1 <= nt <= QS_MAX_TARGETS
 *    targets and nt + nc <= n qubits, all distinct and in [0, n).
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QS_MAX_QUBITS 36
#define QS_MAX_CIRCUIT_QUBITS 62 /* qubit indices of a circuit: [0, 62) */
#define QS_MAX_TARGETS 6
#define QS_MAX_KRAUS 64

typedef enum { QS_C64 = 1, QS_C128 = 2 } qs_dtype;

typedef enum {
    QS_OK = 0,
    QS_E_INVAL = -1,       /* malformed argument (null pointer, bad count, non-finite value) */
    QS_E_RANGE = -2,       /* qubit index out of range or repeated */
    QS_E_NOMEM = -3,       /* allocation failed or above the memory limit */
    QS_E_DEVICE = -4,      /* a HIP runtime call failed */
    QS_E_ZERO_NORM = -5,   /* a Kraus branch or state with zero probability */
    QS_E_UNSUPPORTED = -6  /* valid request that the library does not implement */
} qs_status;

typedef struct qs_state qs_state;     /* opaque */
typedef struct qs_circuit qs_circuit; /* opaque */

/* ---------------------------------------------------------------- state -- */

/* Allocate a 2^n-amplitude state on the current HIP device and initialise it
 * to |0...0> (App. A-1 QINIT).  The state gets its own non-blocking stream of
 * default priority.  Errors: QS_E_INVAL (n, dt or out), QS_E_NOMEM (device
 * allocation failed, or 2^n * sizeof(amplitude) above qs_set_memory_limit). */
qs_status qs_create(int n, qs_dtype dt, qs_state **out);

/* Same as qs_create, but the amplitudes live in a caller-owned device buffer
 * of `bytes` bytes (at least 2^n * sizeof(amplitude), 16-byte aligned), for
 * example a torch tensor's storage, and work is enqueued on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  The buffer must outlive the
 * state; qs_destroy does not free it.  The buffer is initialised to |0...0>. */
qs_status qs_create_from_buffer(int n, qs_dtype dt, void *device_buffer, size_t bytes,
                                void *hip_stream, qs_state **out);

/* Free the state (and its device memory when owned).  NULL is accepted. */
qs_status qs_destroy(qs_state *s);

/* Re-initialise to |0...0> (App. A-1 QINIT). */
qs_status qs_reset(qs_state *s);

/* Overwrite all amplitudes from host memory: 2^n (re, im) double pairs in
 * index order (converted to float for QS_C64).  Synchronous. */
qs_status qs_set_amplitudes(qs_state *s, const double *amps);

/* Number of qubits, dtype, and the device pointer / stream of the state. */
qs_status qs_info(const qs_state *s, int *n, qs_dtype *dt, void **device_ptr, void **hip_stream);

/* Wait for all work enqueued on the state's stream. */
qs_status qs_synchronize(qs_state *s);

/* Upper bound on the bytes one state may allocate (0 = no limit, the
 * default).  Process-wide; lets a caller refuse oversized states up front. */
qs_status qs_set_memory_limit(size_t bytes);

/* ---------------------------------------------------------------- gates -- */

/* Apply a gate: Eq. 2 for one target (the pair (alpha_i, alpha_{i+2^k}) of
 * every i with i_k = 0 is multiplied by the 2x2 matrix), Eq. 3 for controls,
 * and its generalisation to nt <= 6 targets (the 2^nt amplitudes that differ
 * only in the target bits are multiplied by the matrix).  `m` holds 2 * 4^nt
 * doubles as described above; it need not be unitary.  Diagonal matrices and
 * matrices that act as the identity unless some target bit is 1 are
 * recognised and applied by cheaper kernels that touch only the amplitudes
 * they change.  Errors: QS_E_INVAL, QS_E_RANGE. */
qs_status qs_apply_gate(qs_state *s, const int *targets, int nt, const int *controls, int nc,
                        const double *m);

/* Noisy gate of Sec. 2.4: U = `m` on the targets (no controls: nc must be 0,
 * else QS_E_UNSUPPORTED), followed by the Kraus channel {K_b}, b < nk, given
 * in `kraus` as nk matrices of the same layout as `m`, one after another.
 * Branch probabilities are p_b = ||K_b U psi||^2 on the post-gate state,
 * computed in FP64; the branch is the first b with u < p_0 + ... + p_b (if
 * rounding leaves u beyond the total, the last b with p_b > 0); the state
 * becomes K_b U psi / sqrt(p_b).  u in [0, 1) is supplied by the caller.
 * On return *chosen = b and *p_chosen = p_b (either may be NULL).
 * The Kraus set must satisfy sum_b K_b^dagger K_b = I to 1e-10 (Sec. 2.4),
 * else QS_E_INVAL.  QS_E_ZERO_NORM if every p_b is 0.  Synchronises. */
qs_status qs_apply_noisy_gate(qs_state *s, const int *targets, int nt, const int *controls,
                              int nc, const double *m, const double *kraus, int nk, double u,
                              int *chosen, double *p_chosen);

/* ------------------------------------------------------------- circuits -- */

/* A circuit is a flat list of gates and noise sites with DAGGER / CONTROL
 * groups (App. A-1), built by the append calls below and consumed by
 * qs_run_circuit.  Group markers must be balanced when the circuit is run.
 * DAGGER: the group is replaced by the conjugate transposes of its gates in
 * reverse order.  CONTROL q: every gate of the group gains control qubit q.
 * Groups nest.  Noise sites inside a group are QS_E_UNSUPPORTED.  Gate,
 * noise and CONTROL qubits lie in [0, QS_MAX_CIRCUIT_QUBITS) (QS_E_RANGE
 * otherwise), so that circuits wider than any state can be cut by
 * qs_partial_amplitudes; a run on an n-qubit state rejects qubits >= n. */
qs_status qs_circuit_create(qs_circuit **out);
qs_status qs_circuit_destroy(qs_circuit *c);
qs_status qs_circuit_append_gate(qs_circuit *c, const int *targets, int nt, const int *controls,
                                 int nc, const double *m);
/* A Kraus channel on `targets` acting right after the previous gate, which
 * must have the same targets in the same order and no controls: together they
 * form the noisy gate K_b * U of Sec. 2.4.  Noise site s of a run (s = 0, 1, ...
 * in order) draws u = Philox4x32-10 uniform (see qs_philox_uniform) with the
 * run's seed and trajectory. */
qs_status qs_circuit_append_noise(qs_circuit *c, const int *targets, int nt, const double *kraus,
                                  int nk);
qs_status qs_circuit_begin_dagger(qs_circuit *c);
qs_status qs_circuit_end_dagger(qs_circuit *c);
qs_status qs_circuit_begin_control(qs_circuit *c, int qubit);
qs_status qs_circuit_end_control(qs_circuit *c);
/* Counts after group expansion: gates, noise sites, and logical gates (gates
 * whose matrix is not the identity). */
qs_status qs_circuit_counts(const qs_circuit *c, int64_t *gates, int64_t *noise_sites,
                            int64_t *logical_gates);

typedef enum {
    QS_PLAN_UNFUSED = 0,  /* one kernel launch per gate (Eq. 2 / Eq. 3 sweeps) */
    QS_PLAN_GREEDY = 1,   /* gates fused into dense blocks of <= k_max qubits */
    QS_PLAN_LEARNED = 2,  /* fusion partition chosen with the trained cost model */
    QS_PLAN_AUTOTUNE = 3  /* fusion widths chosen by measurement (qs_circuit_autotune_result) */
} qs_plan;

typedef struct {
    int plan;           /* qs_plan */
    int k_max;          /* widest fused block, 1..6 (0 = default) */
    uint64_t seed;      /* Philox key of the noise sites */
    uint64_t traj;      /* trajectory index (Philox counter words 2-3) */
    int64_t *chosen;    /* optional output: Kraus branch of every noise site */
    int64_t chosen_len; /* capacity of `chosen` */
    int tile_qubits;    /* complex64 fused plans: qubits per LDS tile, 10..13 (0 = default) */
    int tile_order;     /* complex64 fused plans: order in which a sweep visits its tiles.
                         * 0 = chosen per sweep by measurement: the first QS_TILE_ORDERS runs of
                         * a plan each use one candidate order for every sweep, timed with HIP
                         * events (those runs synchronise the stream at their end), and later
                         * runs use each sweep's fastest; 1..QS_TILE_ORDERS = that candidate
                         * for every sweep.  Results do not depend on the order. */
    int direct_launch;  /* qs_run_trajectories: 0 = each device-sampled pass runs as one captured
                         * HIP graph; 1 = the same launches enqueued one by one */
} qs_run_opts;

/* Candidate tile orders of a sweep (qs_run_opts.tile_order). */
#define QS_TILE_ORDERS 4

/* Shape of the plan qs_run_circuit would execute for this circuit on an
 * n-qubit state of dtype dt with these options (opts may be NULL): the number
 * of kernel launches that sweep the whole state, the number of fused blocks
 * (dense matrix-core blocks and diagonal passes inside those sweeps, or fused
 * gates of the per-block plan) and the number of logical gates.  Needs no
 * state; with QS_PLAN_LEARNED and an installed cost model the candidate
 * plans are scored on the current device. */
qs_status qs_circuit_plan_info(const qs_circuit *c, int n, qs_dtype dt, const qs_run_opts *opts,
                               int64_t *sweeps, int64_t *blocks, int64_t *logical_gates);

/* Apply every gate and noise site of the circuit to the state, in order
 * (Sec. 2.2, third step: one traversal of the instruction list).  opts may be
 * NULL (= unfused, seed 0, trajectory 0).  Fused plans apply the same
 * operator up to rounding: on complex64 states they run as tile sweeps (a
 * tile of 2^tile_qubits amplitudes in LDS receives a run of fused 4- and
 * 5-qubit blocks on the matrix cores, with split-bfloat16 operands and FP32
 * accumulation, keeping about 16 significant bits per block); on complex128
 * states as one FP64 sweep per fused block.  Noise sites split the circuit
 * into segments: the gates between two sites are planned and fused as one
 * segment, and each site is sampled on the state that the segments before it
 * left (Sec. 2.4).  Synchronises only when the circuit has noise sites.
 * Errors: QS_E_INVAL (unbalanced groups, k_max), QS_E_RANGE (a qubit >= n),
 * QS_E_UNSUPPORTED (noise inside a group). */
qs_status qs_run_circuit(qs_state *s, const qs_circuit *c, const qs_run_opts *opts);

/* Autotuning (QS_PLAN_AUTOTUNE).  The candidates are the fused plans of the
 * state's shape: tile_qubits in {11, 12, 13} (at most n) x k_max in {4, 5}
 * for complex64 states of at least 11 qubits, k_max in {2, 3, 4} otherwise.
 * Each of the first runs of a circuit on a state of a given (n, dtype) takes
 * the next untried candidate and times its execution on the state's stream
 * (planning and the upload of its operand program excluded; the call then
 * synchronises); once every candidate has run, later runs use the fastest.
 * Every run is a complete, exact execution of the circuit.  Tuning records
 * belong to the circuit and are cleared when it changes.
 * qs_circuit_autotune_result reports, for (n, dt): the number of candidates
 * tried so far, the number of candidates, and the fastest one (tile_qubits = 0
 * for per-block plans) with its time in seconds (all 0 before any run). */
qs_status qs_circuit_autotune_result(const qs_circuit *c, int n, qs_dtype dt, int *tried, int *candidates,
                                     int *tile_qubits, int *k_max, double *seconds);

/* ------------------------------------------------------------- readout -- */

/* Copy amplitudes to the host as (re, im) doubles: out[2k], out[2k+1] =
 * alpha_{idx[k]} for k < m; idx == NULL means all 2^n amplitudes in index
 * order (m must then be 2^n).  Indices >= 2^n are QS_E_RANGE. */
qs_status qs_amplitudes(const qs_state *s, const uint64_t *idx, size_t m, double *out);

/* PMEASURE (App. A-1): probabilities of the 2^nq outcomes of the listed
 * qubits, accumulated in FP64; bit (nq-1-b) of the outcome index is the
 * value of qubits[b] (first listed = most significant, as in the output of
 * App. A-2).  qubits == NULL means all n qubits in the order n-1, ..., 0, so
 * that out[i] = |alpha_i|^2.  The state is unchanged.  nq <= 30. */
qs_status qs_probabilities(const qs_state *s, const int *qubits, int nq, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * PMEASURE probabilities of qs_probabilities, computed by the same kernels,
 * for a state held in caller-owned device memory, written to caller-owned
 * device memory.  device_amps: 2^n amplitudes of dtype dt as a state stores
 * them (16-byte aligned), only read; qubits / nq as in qs_probabilities
 * (NULL = all n qubits, n-1 first); device_out: 2^nq doubles (8-byte
 * aligned), only written.  Work is enqueued on hip_stream (a hipStream_t;
 * NULL = the default stream) and the call returns without waiting; it
 * makes no allocation of any kind (no hipMalloc, no host allocation).  The
 * block partial sums live in a static device array of
 * QS_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; every call
 * on one GPU shares it and overwrites what it reads (nothing needs to start
 * at zero), so calls that overlap in time on one GPU race: order them on one
 * stream.  Errors: QS_E_INVAL (pointers, alignment, n, dt, nq), QS_E_RANGE
 * (qubits, or a reduction needing more than the static scratch),
 * QS_E_UNSUPPORTED (nq > 30), QS_E_DEVICE. */
#define QS_NOALLOC_SCRATCH_BYTES (8u * 1024u * 1024u + 512u)
qs_status qs_probabilities_noalloc(const void *device_amps, int n, qs_dtype dt, const int *qubits, int nq,
                                   double *device_out, void *hip_stream);

/* Squared norm sum_i |alpha_i|^2, accumulated in FP64. */
qs_status qs_norm(const qs_state *s, double *out);

/* <Z_q> = sum_i |alpha_i|^2 (1 - 2 i_q) for every qubit q < n, in FP64. */
qs_status qs_expect_z(const qs_state *s, double *out);

/* ----------------------------------------------------- noisy trajectories -- */

/* Run `count` independent noisy trajectories (Sec. 2.4): trajectory t
 * evolves a state of widths[t] qubits (1..36) from |0...0> under circs[t]
 * with Philox trajectory index t and key `seed` (noise sites drawn as in
 * qs_run_circuit), then writes its <Z_q> for q < widths[t] to z_out at
 * offset sum_{t' < t} widths[t'].  Noise sites must have state-independent
 * branch weights (every K_b^dagger K_b a multiple of I: flips,
 * depolarizing; drawn on the host before any launch) or be damping-type
 * one-qubit channels (K1 = diag(1, k), K2 nonzero only in column 1:
 * amplitude and phase damping), whose weights come from FP64 prefix sums
 * of the state.  All states live in one device allocation.
 * Complex64 states of at least 10 qubits run in device-sampled passes: all
 * remaining steps of all trajectories are planned as tile sweeps, uploaded
 * once and executed as one captured HIP graph (opts->direct_launch = 0) of
 * batched sweeps, batched FP64 run sums and a sampling kernel that draws
 * each damping site's uniform on the device and picks its branch.  A
 * trajectory whose site takes K2 stops there; once its job has finished,
 * the host rewrites its remaining steps (K1 of the earlier sites of the run,
 * K2, renormalisation, the rest of the run) and queues it for the next job.  Complex128 states, narrower states and plans with gates too
 * wide for a tile take the host-sampled path (one batched step at a time,
 * sums read back and sampled on the host); so does every state with
 * opts->plan = QS_PLAN_UNFUSED.  Device-sampled trajectories run in jobs of
 * at most 128, launched so that the host plans one job while the device runs
 * the one before.  opts (may be NULL): plan QS_PLAN_GREEDY (default widths:
 * 13-qubit tiles, 4-qubit blocks, 1 outer selector bit per op, 128
 * trajectories per job) or QS_PLAN_AUTOTUNE (each of the first calls for a batch of the same
 * dtype, size and widths runs the next untried candidate width set and
 * times the whole call; a call that had to enlarge the job buffers kept
 * between calls is not recorded and its candidate runs again; later calls
 * use the fastest: qs_trajectory_stats reports the choice), k_max (4 or 5; 0 = default), tile_qubits (10..13;
 * 0 = default), direct_launch.  The branch choices do not depend on any of
 * these.  *traj_per_s (may be NULL) receives count / the wall time of the
 * whole call after argument checks: preparation of every trajectory,
 * planning, device allocation, uploads, all launches and the final
 * reductions.  Synchronous.  The job buffers (device program and work
 * space, pinned host staging) stay allocated after the call, one set per
 * device, and are reused by the next call.  Errors: QS_E_INVAL (arguments, widths),
 * QS_E_RANGE (a qubit >= the trajectory's width), QS_E_UNSUPPORTED (noise
 * inside a group, or a channel of another form), QS_E_ZERO_NORM,
 * QS_E_NOMEM, QS_E_DEVICE. */
qs_status qs_run_trajectories(const qs_circuit *const *circs, const int *widths, int count,
                              qs_dtype dt, uint64_t seed, const qs_run_opts *opts, double *z_out,
                              double *traj_per_s);

/* Statistics of the last qs_run_trajectories call on the calling thread. */
typedef struct {
    int passes;             /* the most device-sampled jobs one trajectory ran in (more than one: it jumped) */
    int graphs;             /* device-sampled jobs (each one HIP graph, or one set of launches) */
    int chunk;              /* trajectories per job at most (0 = all waiting trajectories in one job) */
    int host_sampled;       /* trajectories that took the host-sampled path */
    int64_t jumps;          /* K2 branches taken */
    int64_t launches;       /* kernel launches enqueued (inside graphs included) */
    int graph;              /* 1 when the passes ran as captured HIP graphs */
    int tile_qubits;        /* widths used: qubits per tile (at most the state's width), */
    int k_max;              /*   widest fused block, */
    int max_outer;          /*   outer selector bits per tile op */
    int autotune_tried;     /* QS_PLAN_AUTOTUNE: candidates measured so far for this batch shape */
    int autotune_candidates;
    double seconds;         /* wall time of the call */
    double host_seconds;    /* of which: trajectory preparation, planning, program build and upload of the jobs (host) */
    double device_seconds;  /* device time of the jobs (HIP events around each) */
} qs_traj_stats;

qs_status qs_trajectory_stats(qs_traj_stats *out);

/* ------------------------------------------------------- sharded states -- */

#define QS_REMAP_MAX_G 10

/* Qubit-remap exchange, the device-local halves.  Sec. 2.1 divides the
 * amplitudes of a state equally over the nodes, so the top g qubits of an
 * (L + g)-qubit state name the node (here: the device) holding an
 * amplitude, and each device keeps a shard of L local qubits in a qs_state.
 * A gate on a global qubit needs partner amplitudes held elsewhere, the slow
 * case of Sec. 3.1 / Fig. 4.  Instead of exchanging pairs per gate, the g
 * global qubits swap places with g local qubits lq[0..g-1] (distinct, in
 * [0, L)) in one all-to-all, which the caller runs between these calls
 * (for example RCCL's all-to-all on the state's stream):
 *  - qs_remap_pack writes the shard into `device_buf` as 2^g chunks of
 *    2^(L-g) amplitudes, chunk d (at offset d * 2^(L-g) amplitudes) holding
 *    the amplitudes whose bits lq read d (bit i of d = local qubit lq[i]),
 *    in ascending order of the remaining local bits.  The shard is unchanged.
 *  - chunk d of device r goes to slot r of device d's receive buffer;
 *  - qs_remap_unpack overwrites the shard from such a buffer, slot r going
 *    to the amplitudes whose bits lq read r.
 * Afterwards local qubit lq[i] carries the former global qubit L + i and
 * global qubit L + i the former local qubit lq[i]; with g = 0 both calls
 * are plain copies.  `device_buf`: caller-owned device memory of at least
 * 2^L amplitudes of the state's dtype, 16-byte aligned, not overlapping the
 * state; only read by unpack, only written by pack.  Both calls are
 * enqueued on the state's stream and return before the device finishes.
 * Errors: QS_E_INVAL (null pointer, misaligned buffer, g outside
 * [0, min(L, QS_REMAP_MAX_G)], buffer overlapping the state), QS_E_RANGE
 * (lq repeated or outside [0, L)), QS_E_DEVICE. */
qs_status qs_remap_pack(const qs_state *s, int g, const int *lq, void *device_buf);
qs_status qs_remap_unpack(qs_state *s, int g, const int *lq, const void *device_buf);

/* ------------------------------------------------- partial-amplitude mode -- */

#define QS_PARTIAL_MAX_CUTS 24

/* Partial-amplitude mode (Sec. 2.2 (partial), Eq. 4, Fig. 1): amplitudes of
 * an n-qubit circuit (2 <= n <= 62) from sub-circuits on two parts of the
 * qubits, never holding a 2^n state.  Part A is the qubits whose bits are set
 * in part_a, part B the others; each part is renumbered in ascending qubit
 * order and may hold at most QS_MAX_QUBITS qubits.  Gates inside one part
 * belong to that part's sub-circuit.  A gate crossing the dividing line is
 * cut as Eq. 4 cuts CZ when, in canonical form (a target on which the matrix
 * is the identity unless its bit is 1 becomes a control; diagonal matrices
 * are phase gates), it is
 *  - a dense gate whose targets lie in one part: its controls in the other
 *    part (at most QS_MAX_TARGETS) become a projector there, onto all ones
 *    (branch 1, the gate applied under its remaining controls) or onto the
 *    rest (branch 0, no gate); CNOT, CU3 and Toffoli are cut this way;
 *  - a phase gate with exactly one qubit in one part and at most
 *    QS_MAX_TARGETS in the other: the projector P_0 or P_1 on that qubit and
 *    the matching diagonal factor on the others (CZ, CR).
 * Every cut doubles the circuits (Sec. 2.2 (partial), first step).  For each
 * branch word w < 2^c (bit j = branch of cut j, cuts in circuit order) the
 * two sub-circuits run from |0...0> on states of n_A and n_B qubits, as
 * qs_run_circuit runs them with `opts` (NULL = unfused; QS_PLAN_AUTOTUNE is
 * not accepted), and amp(x) = sum_w psiA_w(x_A) psiB_w(x_B), with x_A / x_B
 * the bits of x in part A / B, accumulated in FP64 on the device (last
 * step).  The gates of a part between two cuts do not depend on later
 * branches, so when c + 1 states of each part fit in 32 GiB (and in the
 * qs_set_memory_limit bound) the branch words are walked depth first and
 * each segment between cuts runs once per prefix, from a copy of the state
 * before it; otherwise each branch word runs both sub-circuits in full.
 * out[2k], out[2k+1] = amp(idx[k]) for k < m; *cuts (may be NULL)
 * receives c.  Synchronous.  Errors: QS_E_INVAL (pointers, n, part_a, dt,
 * opts), QS_E_RANGE (a gate qubit >= n, an index >= 2^n), QS_E_UNSUPPORTED
 * (noise sites, a crossing gate of another form, more than
 * QS_PARTIAL_MAX_CUTS cuts, a part wider than QS_MAX_QUBITS), QS_E_NOMEM,
 * QS_E_DEVICE. */
qs_status qs_partial_amplitudes(const qs_circuit *c, int n, qs_dtype dt, uint64_t part_a, const uint64_t *idx,
                                size_t m, double *out, const qs_run_opts *opts, int *cuts);

/* The number of cuts qs_partial_amplitudes makes for this circuit and
 * division (host only, no device work); errors as qs_partial_amplitudes. */
qs_status qs_partial_cuts(const qs_circuit *c, int n, uint64_t part_a, int *cuts);

/* ------------------------------------------------- single-amplitude mode -- */

#define QS_SINGLE_MAX_SLICES 16

/* Shape of a single-amplitude contraction (Sec. 2.3). */
typedef struct {
    int vertices;       /* Boolean variables of the graphical model (Fig. 2): one per qubit at the
                         * start and one per target of every gate that is not diagonal */
    int tensors;        /* edges: one per non-identity gate, plus a vector of ones for every vertex
                         * that ends up on a single edge */
    int fixed;          /* vertices fixed: initial state, measured bits, slices */
    int sliced;         /* vertices fixed by slicing: 2^sliced graphs per amplitude */
    int merges;         /* pairwise tensor merges (one device launch each) */
    int max_rank;       /* indices of the largest merged tensor */
    double flops;       /* real FP64 flops of the merges for one amplitude (all slices) */
    double peak_bytes;  /* device arena of the tensors (qs_single_plan: one bitstring) */
    int batch;          /* graphs contracted side by side per launch (bitstrings x slices) */
    int own_low;        /* merge operands stored with their own vertices lowest (the others: the
                         * summed vertices lowest), chosen so that merges write whole lines */
} qs_single_info;

/* Single-amplitude mode (Sec. 2.3, Figs. 2-3): amplitudes <x|C|0...0> of an
 * n-qubit unitary circuit (1 <= n <= 62), never holding a 2^n state.  The
 * circuit is mapped to an undirected graphical model: a vertex per Boolean
 * variable, an edge (tensor) per gate; a diagonal gate keeps its qubits'
 * vertices, any other gate gives each target a new vertex (controls are kept),
 * and a gate's tensor over (new target vertices, old target vertices,
 * controls) holds U[new, old] where every control is 1 and delta(new, old)
 * elsewhere.  Each qubit's first vertex is fixed to 0 and its last to bit q
 * of x; the nslice free vertices on the most edges are fixed to every
 * combination of values, giving 2^nslice graphs (differential elimination).
 * All other vertices are eliminated one by one, the next chosen as the one
 * whose merged tensor is smallest: the tensors on it are merged in order of
 * rank and the vertex summed out with the last merge (integral
 * elimination).  The merges run on the device as batched complex FP64
 * contractions (all bitstrings of a chunk and all slices side by side); the
 * product of the remaining scalars, summed over the slices, is the
 * amplitude.  bits[k] holds x for k < m (bit q = measured value of qubit q);
 * out[2k], out[2k+1] = the amplitude.  nslice in [0, QS_SINGLE_MAX_SLICES]
 * does not change the result (up to rounding).  info (may be NULL) receives
 * the shape.  Bitstrings are processed in chunks whose tensors fit 64 GiB
 * (and the qs_set_memory_limit bound).  Synchronous.  Errors: QS_E_INVAL
 * (pointers, n, nslice), QS_E_RANGE (a gate qubit >= n, a bitstring with a
 * bit >= n), QS_E_UNSUPPORTED (noise sites), QS_E_NOMEM (one bitstring's
 * tensors do not fit), QS_E_DEVICE. */
qs_status qs_single_amplitudes(const qs_circuit *c, int n, const uint64_t *bits, size_t m, int nslice,
                               double *out, qs_single_info *info);

/* The shape qs_single_amplitudes would contract for one bitstring (host only,
 * no device work); errors as qs_single_amplitudes. */
qs_status qs_single_plan(const qs_circuit *c, int n, int nslice, qs_single_info *info);

/* --------------------------------------------------------------- scripts -- */

/* Input scripts in the instruction set of App. A-1, one instruction per line
 * (names case-insensitive, arguments separated by commas, angle arguments
 * optionally in double quotes as App. A-2 prints them: a number, pi, or an
 * expression of them with + - * / and parentheses; '#' starts a comment and
 * lines starting with '%' are section labels):
 *   QINIT n | CREG m | H/X/Y/Z/S/T i | RX/RY/RZ i, theta | U4 i, a, b, c, d
 *   (the angle form) | CNOT/CZ i, j | CR i, j, theta | SWAP/ISWAP i, j |
 *   TOFFOLI i, j, k | DAGGER ... ENDDAGGER | CONTROL i ... ENDCONTROL [i] |
 *   MEASURE i, $j | PMEASURE i, j, ..., k
 * with the matrices of App. A-1 (controlled gates act on the last listed
 * qubit when the others are 1).  MEASURE i, $j is a projective measurement
 * of qubit i in the computational basis: a noise site with the Kraus set
 * {|0><0|, |1><1|} after an identity gate, so the outcome b is drawn as in
 * Sec. 2.4 (p_b = ||P_b psi||^2 in FP64, the run's Philox draw, the state
 * renormalised) and stored in classical register j.  PMEASURE changes no
 * state and must come after every other operation; at most one per script.
 * QINIT comes first; qubit and register numbers are checked against it and
 * CREG.  qs_script_parse builds a new circuit (freed by the caller with
 * qs_circuit_destroy) and fills `info`; it needs no device.  Errors name the
 * line: QS_E_INVAL (syntax, unknown instruction, missing QINIT, unbalanced
 * groups, PMEASURE not last), QS_E_RANGE (qubit or register numbers),
 * QS_E_UNSUPPORTED (MEASURE inside a DAGGER / CONTROL group). */
typedef struct {
    int n;            /* QINIT */
    int creg;         /* CREG (0 when absent) */
    int measures;     /* MEASURE instructions */
    int pmeasure_n;   /* qubits listed by PMEASURE (0 when absent) */
    int pmeasure[QS_MAX_QUBITS];
} qs_script_info;

qs_status qs_script_parse(const char *text, qs_circuit **circuit, qs_script_info *info);

/* Parse and run a script on a new n-qubit state of dtype dt, from |0...0>
 * (QINIT), with Philox key `seed` and trajectory 0 for the MEASURE draws,
 * per-gate launches when it measures, else `plan` (a qs_plan value; not
 * QS_PLAN_AUTOTUNE).  creg[j] (creg_len >= CREG entries) receives the last
 * outcome stored in register j (0 if none); probs (probs_len >= 2^pmeasure_n
 * doubles) the PMEASURE probabilities in the order of qs_probabilities.
 * Either output may be NULL when the script has no such instruction; info
 * may be NULL.  Synchronous.  Errors as qs_script_parse and qs_run_circuit,
 * QS_E_INVAL for short outputs. */
qs_status qs_script_run(const char *text, qs_dtype dt, uint64_t seed, int plan, int *creg, int creg_len,
                        double *probs, size_t probs_len, qs_script_info *info);

/* ------------------------------------------------------------------ misc -- */

/* The uniform number used for noise site `site` of trajectory `traj`:
 * Philox4x32-10 (Salmon et al., SC'11) with counter (site lo, site hi,
 * traj lo, traj hi) and key (seed lo, seed hi); the first two output words
 * form x = w1 * 2^32 + w0 and u = (x >> 11) * 2^-53 in [0, 1). */
double qs_philox_uniform(uint64_t seed, uint64_t traj, uint64_t site);

/* Philox4x32-10 block function itself (counter[4], key[2] -> out[4]). */
void qs_philox4x32_10(const uint32_t *counter, const uint32_t *key, uint32_t *out);

/* Kernel timing.  While enabled, every launch on the state's stream is
 * bracketed by HIP events.  qs_profile_query synchronises and returns, for
 * kernel class `kernel` (qs_kernel_class), the number of launches, their
 * summed device time in ms and their summed algorithmic bytes and flops
 * (the bytes the method must move: read + write of every amplitude the
 * launch changes; reductions read every amplitude once). */
typedef enum {
    QS_K_INIT = 0,
    QS_K_DENSE1 = 1,  /* one target, Eq. 2 / Eq. 3 */
    QS_K_DENSE2 = 2,  /* two targets */
    QS_K_DENSE3 = 3,  /* three targets */
    QS_K_DENSEN = 4,  /* four to six targets, FP64/FP32 vector units */
    QS_K_PHASE = 5,   /* diagonal gates */
    QS_K_FUSED = 6,   /* fused dense block on matrix cores */
    QS_K_TILE = 7,    /* multi-gate tile sweep */
    QS_K_REDUCE = 8,  /* FP64 reductions */
    QS_K_OTHER = 9,
    QS_K_COUNT = 10
} qs_kernel_class;

qs_status qs_profile_enable(qs_state *s, int on);
qs_status qs_profile_reset(qs_state *s);
qs_status qs_profile_query(qs_state *s, int kernel, int64_t *launches, double *total_ms,
                           double *alg_bytes, double *alg_flops);

/* --------------------------------------------------------- cost model -- */

/* The learned fusion planner scores candidate tile plans with a small fully
 * connected network F -> H -> H -> 1 (ReLU, FP32; H must be 64), trained on
 * the simulator's own timings of tile sweeps.  Parameters are packed as
 * W1[H][F], b1[H], W2[H][H], b2[H], W3[H], b3 (float); the loss is the mean
 * squared error.  All compute runs on the current device; host arrays are
 * copied in and out.  Not in the paper: a planning aid of this library. */
#define QS_COST_FEATURES 16

/* y[i] = network(x[i * f .. i * f + f)) for i < n. */
qs_status qs_mlp_forward(const float *params, int f, int h, const float *x, int64_t n, float *y);

/* Mean squared-error loss over the n samples and its exact gradient
 * (same packing as params). */
qs_status qs_mlp_grad(const float *params, int f, int h, const float *x, const float *t, int64_t n,
                      float *loss, float *grad);

/* `steps` Adam steps (beta 0.9 / 0.999) with learning rate lr on minibatches
 * of `batch` samples drawn with replacement (Philox, key `seed`); params are
 * updated in place; *loss receives the last minibatch loss. */
qs_status qs_mlp_train(float *params, int f, int h, const float *x, const float *t, int64_t n, int steps,
                       int batch, float lr, uint64_t seed, float *loss);

/* Training samples recorded while profiling is enabled: one per tile sweep,
 * QS_COST_FEATURES features (tile size, state size, dense blocks of 4 and 5
 * qubits, diagonal passes, outer selector bits, identity-skips, gates, the six
 * highest tile qubits, dtype, matrix-core work) and the target
 * ln(sweep time in ns / 2^n).  Copies up to `capacity` samples, removes them
 * from the state, and sets *count. */
qs_status qs_profile_samples(qs_state *s, float *features, float *log_ns_per_amp, int64_t capacity,
                             int64_t *count);

/* Install trained parameters (f = QS_COST_FEATURES, h = 64) for
 * QS_PLAN_LEARNED; NULL removes the model (the greedy plan is then used). */
qs_status qs_cost_model_set(const float *params, int f, int h);

/* Text of the last error on this thread ("" if none).  Valid until the next
 * failing call on the same thread. */
const char *qs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
