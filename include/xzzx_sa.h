/*
 * xzzx_sa.h -- C ABI of the MI355X (gfx950) simulated-annealing decoder for the
 * XZZX surface code under Y-biased code-capacity noise (arXiv:2509.17837).
 *
 * The decoder follows Alg. 7 of the paper: randomized greedy matching
 * (Alg. 6) gives one reference configuration R_r per replica r; every replica
 * runs four annealing chains, one per logical coset (Alg. 2, Metropolis moves
 * of Alg. 3 that multiply by one stabilizer generator); the minimum energy per
 * coset (Eqs. (18)-(21)) selects the logical class P*, and the minimum-energy
 * configuration found is returned as the recovery.
 *
 * Conventions
 *   Pauli codes (footnote to Eq. (10)): upper bit X, lower bit Z:
 *     I=0, Z=1, X=2, Y=3; one uint8_t per qubit.  Products are XOR.
 *   Logical class indices: I=0, X=1, Y=2, Z=3 (loop order of Alg. 1),
 *     always relative to the replica-0 reference R_0 (the paper's R_1).
 *   Energies: int32 sums of integer weights W[code] = round(2^16 * -ln(p_P/(1-p)))
 *     (Eqs. (8)-(12)); 2^16 units = 1 nat, so beta = 1 is the Nishimori point.
 *   Chains: chain c = 4r + P' of a syndrome starts at R_r * L_P' (Eq. (36)).
 *   Random numbers: Philox4x32-10.  Greedy tie key of pair id k of colour g in
 *     replica r of syndrome uid: word 0 of Philox(greedy_seed; uid, r,
 *     0x100+g, k).  Metropolis draw of generator rank m in colour class kc in
 *     sweep t of chain c: word (m mod 4) of Philox(anneal_seed; uid, c,
 *     4t+kc, m div 4).
 *   Acceptance (Alg. 3): dE <= 0, or u < ceil(2^32 exp(-beta[t] dE 2^-16))
 *     with that threshold clamped to 2^32-1.
 *   E_min (Alg. 2) is taken after each colour class of each sweep; "stop"
 *     4t+kc+1 names the first phase attaining it (0 = initial configuration).
 *
 * Memory and ownership
 *   Pointers named d_* are device pointers (HIP device memory of the current
 *   device); every other pointer is host memory.  The caller allocates and
 *   owns every data buffer and the workspace; the library never frees them.
 *   Handles (lattice, plan, graph, server) are created and destroyed only
 *   through this API.  Host inputs are copied before the call returns.
 *   Device work is enqueued on the given hipStream_t (passed as void*, NULL =
 *   the null stream); outputs are valid once that stream has completed.
 *
 * Errors
 *   Every int-returning call returns XZZX_OK (0) or a negative status; on
 *   failure outputs are undefined and xzzx_last_error() returns a message
 *   (thread-local).  No C++ exception crosses this interface.
 *
 * Thread safety and streams
 *   Calls on distinct handles may run concurrently.  A plan may be used by
 *   several concurrent decode, anneal or graph-capture calls on different
 *   streams: a call that runs launches concurrently does so on side streams
 *   of its own caller stream (created on first use, kept until the process
 *   ends), so calls on different streams share no internal stream and a
 *   capture on one stream never records another call's work.  (xzzx_graph_create
 *   creates them before it begins capturing; a caller capturing a decode in
 *   its own graph in global capture mode makes one call on that stream first,
 *   or uses xzzx_decode_noalloc, which creates none.)  The plan
 *   setters (set_lanes, set_kernel, set_order, set_ladder, autotune) change
 *   what later calls launch, and set_ladder replaces device tables: none may
 *   run while a call that uses the plan is being enqueued or its work is in
 *   flight (synchronise those streams first).  Server submit/poll are
 *   thread-safe; other calls on one handle need external synchronisation.
 */
#ifndef XZZX_SA_H
#define XZZX_SA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    XZZX_OK = 0,
    XZZX_EINVAL = -1,   /* bad argument */
    XZZX_ENOMEM = -2,   /* allocation failed or workspace too small */
    XZZX_EDEVICE = -3,  /* HIP runtime error */
    XZZX_ERANGE = -4,   /* energies or tables would overflow their integer types */
    XZZX_EAGAIN = -5,   /* server over budget; retry later */
    XZZX_ENOTREADY = -6 /* result not yet available */
};

enum { XZZX_ROTATED = 0, XZZX_PLANAR = 1 };
enum { XZZX_BIAS_RATIO = 0, XZZX_BIAS_PAPER = 1 };
enum { XZZX_SCHED_LINEAR = 0, XZZX_SCHED_GEOMETRIC = 1, XZZX_SCHED_PAPER_LOG = 2 };
enum { XZZX_GREEDY_RANDOM = 0, XZZX_GREEDY_SAME = 1, XZZX_GREEDY_BOUNDARY = 2 };

/* decode flags */
enum {
    XZZX_FLAG_PLAIN = 1,         /* one anneal launch per syndrome, no persistent queue */
    /* Stage selection (none set = all stages).  Stages communicate through the
     * workspace, so a split decode passes the same groups and workspace to
     * each call, in this order. */
    XZZX_FLAG_STAGE_GREEDY = 2,  /* greedy references and their classes */
    XZZX_FLAG_STAGE_ANNEAL = 4,  /* annealing of every chain */
    XZZX_FLAG_STAGE_FINISH = 8   /* per-syndrome reduction and recovery */
};

typedef struct xzzx_lattice xzzx_lattice;
typedef struct xzzx_plan xzzx_plan;

/* Message for the last failing call on this thread ("" if none). */
const char *xzzx_last_error(void);

/* ABI version, currently 1. */
int xzzx_version(void);

/* ---- code model (Sec. II) ------------------------------------------------ */

/* Lattice of odd distance 3 <= d <= 31.
 *   XZZX_ROTATED: d^2 qubits, d^2-1 generators; qubit (x,y) has index y*d+x;
 *     cell (i,j), -1 <= i,j <= d-1, holds X(i,j) Z(i+1,j) Z(i,j+1) X(i+1,j+1)
 *     (Eq. (1)); every bulk cell is a generator, boundary cells alternate
 *     (bottom j=-1: i odd; top j=d-1: i even; left i=-1: j even;
 *     right i=d-1: j odd).  Generators are numbered row-major over (j,i).
 *   XZZX_PLANAR: the paper's lattice, d^2+(d-1)^2 qubits, 2d(d-1) generators
 *     (Sec. II, Sec. IV.B.1), generators numbered row-major in doubled
 *     coordinates.
 * Returns EINVAL for an unknown layout or an even/out-of-range d. */
int xzzx_lattice_create(int layout, int d, xzzx_lattice **out);
void xzzx_lattice_destroy(xzzx_lattice *lat);

/* Sizes: qubits, generators, generators per colour class (= n_stabs/4). */
int xzzx_lattice_info(const xzzx_lattice *lat, int *n_qubits, int *n_stabs, int *per_class);

/* Generator tables (host arrays, any may be NULL): face_qubits[n_stabs][4]
 * qubit on the X_left, Z_up, Z_down, X_right slots or -1; face_paulis
 * [n_stabs][4] their codes (2, 1, 1, 2; 0 if absent); face_class (0..3,
 * generators of one class share no qubit); face_colour (decoding-graph colour,
 * Sec. III); face_rank (rank inside the class). */
int xzzx_lattice_tables(const xzzx_lattice *lat, int32_t *face_qubits, uint8_t *face_paulis,
                        int32_t *face_class, int32_t *face_colour, int32_t *face_rank);

/* Logical representatives L_X (top-bottom) and L_Z (left-right), [n_qubits]. */
int xzzx_lattice_logicals(const xzzx_lattice *lat, uint8_t *lx, uint8_t *lz);

/* ---- noise, weights, schedules (Eqs. (5)-(12), (23)-(24)) ----------------- */

/* convention XZZX_BIAS_RATIO (eta = p_Y / (p_X + p_Z)): p_Y = p eta/(eta+1),
 * p_X = p_Z = p/(2(eta+1));
 * XZZX_BIAS_PAPER: p_x:p_y:p_z = 1:eta:1 (Sec. V.A).  pxyz = (p_X, p_Y, p_Z).
 * EINVAL unless 0 < p < 1/2 and eta > 0. */
int xzzx_noise(double p, double eta, int convention, double pxyz[3]);

/* w[4] by code (I,Z,X,Y) = llround(2^16 * -ln(p_P/(1-p))), w[0] = 0;
 * wg[2] = greedy edge weights for X and Z components,
 * llround(2^16 * -ln((p_X+p_Y)/(1-p))) and likewise with p_Z+p_Y (Eq. (27)). */
int xzzx_weights(double p, const double pxyz[3], int32_t w[4], int32_t wg[2]);

/* beta[n] in nats: LINEAR b0..b1 and GEOMETRIC b0..b1 include both ends;
 * PAPER_LOG is Eqs. (23)-(24): b0 (1 + gamma ln i), i = 1..n,
 * gamma = (b1/b0 - 1)/ln n (0 for n < 2). */
int xzzx_schedule(int kind, double b0, double b1, int n, double *beta);

/* Logical class (0..3) of a*b for host configurations with equal syndromes,
 * via commutation with L_X and L_Z (Alg. 7); *cls = -1 if the syndromes
 * differ. */
int xzzx_class_host(const xzzx_lattice *lat, const uint8_t *a, const uint8_t *b, int *cls);

/* ---- plans ---------------------------------------------------------------- */

/* A plan holds, on the current device, everything the kernels need for one
 * (lattice, w, wg, beta schedule): generator descriptors, the dE lookup, the
 * acceptance-threshold table [n_sweeps][distinct dE], logicals and the
 * greedy-matching distance tables (Eqs. (25)-(30)).  beta is copied.
 * ERANGE if n_qubits * max(w) >= 2^31.  n_sweeps may be 0. */
int xzzx_plan_create(const xzzx_lattice *lat, const int32_t w[4], const int32_t wg[2],
                     const double *beta, int n_sweeps, xzzx_plan **out);
void xzzx_plan_destroy(xzzx_plan *plan);

/* Plan facts (any pointer may be NULL): sizes, number of distinct move
 * energies, lanes per chain of the byte-state kernel, and the annealing kernel
 * in use (XZZX_KERNEL_ROWS, XZZX_KERNEL_ROWS_GENERIC, XZZX_KERNEL_BYTES, or
 * XZZX_KERNEL_SITE for the random-site order). */
int xzzx_plan_info(const xzzx_plan *plan, int *n_qubits, int *n_stabs, int *n_sweeps,
                   int *n_dE, int *lanes_per_chain, int *kernel);

/* Result-invariant tuning knob of the byte-state kernel: lanes of a wavefront
 * cooperating on one chain (1, 2, 4, ..., 64); chains per wavefront =
 * 64 / lanes.  A non-zero value also selects that kernel; 0 restores the
 * built-in choice (and the default kernel). */
int xzzx_plan_set_lanes(xzzx_plan *plan, int lanes_per_chain);

/* Which annealing kernel a plan uses (results are identical):
 *   XZZX_KERNEL_ROWS: one chain per lane, 2-bit codes packed row by row;
 *     a variant specialised to the distance keeps every row in registers
 *     and its generator schedule in the instruction stream: rotated lattices
 *     with d <= 31 (batch groups whose 4 n_rep chains per syndrome are not a
 *     multiple of 64 run the generic variant instead, d <= 29, or the
 *     byte-state kernel, d = 31), and planar lattices with d <= 15 (turned
 *     by 45 degrees, any n_rep);
 *   XZZX_KERNEL_ROWS_GENERIC: the packed-row kernel without that
 *     specialisation (rows in LDS, schedule read from the plan): rotated
 *     d <= 29, and planar d <= 15, whose lattice turned by 45 degrees has the
 *     same 2 x 2 generator blocks (rows of 2d + 1 columns);
 *   XZZX_KERNEL_BYTES: byte-per-qubit states, lanes_per_chain lanes per chain;
 *   XZZX_KERNEL_AUTO (the default): ROWS where it applies, else on rotated
 *     lattices ROWS_GENERIC where it applies, else BYTES (on planar lattices
 *     BYTES measured faster than ROWS_GENERIC at d = 9).
 * EINVAL for ROWS or ROWS_GENERIC on a lattice they do not cover.
 * xzzx_plan_info reports ROWS only where the specialised variant runs. */
enum { XZZX_KERNEL_AUTO = 0, XZZX_KERNEL_ROWS = 1, XZZX_KERNEL_BYTES = 2, XZZX_KERNEL_ROWS_GENERIC = 3,
       XZZX_KERNEL_SITE = 4, XZZX_KERNEL_LADDER = 5 };
int xzzx_plan_set_kernel(xzzx_plan *plan, int kernel);

/* Step order of the Metropolis chains (Algs. 2-3).
 *   XZZX_ORDER_COLOUR (default): a sweep visits every generator once, colour
 *     class by colour class (generators of one class act on disjoint qubits);
 *     E_min is updated after each class; chain_stop counts phases 4t + k + 1.
 *   XZZX_ORDER_RANDOM_SITE: Alg. 3 as printed: each of the N_stab steps of
 *     sweep t picks one generator uniformly at random and E_min is updated
 *     after every step.  Step m draws the Philox block (uid, chain,
 *     2^31 + t, m div 2); words 2 (m mod 2) and 2 (m mod 2) + 1 are the site
 *     draw u (generator floor(u N_stab / 2^32) in face-id order) and the
 *     acceptance draw.  chain_stop counts steps t N_stab + m + 1 (0 = the
 *     start).  One chain per lane (XZZX_KERNEL_SITE); the kernel knobs do not
 *     apply, the autotuner leaves the plan unchanged and the serving loop
 *     rejects such plans (EINVAL).
 * The two orders give different, equally valid chains.  EINVAL for an unknown
 * order; ERANGE if n_sweeps * n_stabs >= 2^31 or 64 random-site chains do not
 * fit in 64 KiB of LDS. */
enum { XZZX_ORDER_COLOUR = 0, XZZX_ORDER_RANDOM_SITE = 1 };
int xzzx_plan_set_order(xzzx_plan *plan, int order);

/* Replica exchange (parallel tempering; the paper names it as future work,
 * Sec. VII) instead of the annealing schedule.  levels = K in {1, 2, 4, 8,
 * 16} turns it on, 0 off.  Replicas come in ladders of K consecutive
 * replicas r = bK + j that share the greedy reference of replica b (n_rep of
 * every group must be a multiple of K, else EINVAL at decode).  For each
 * coset P the ladder's chains 4(bK + j) + P run at fixed levels
 * beta_k = beta_lo + k (beta_hi - beta_lo)/(K - 1) (beta_lo when K = 1),
 * chain j starting at level j; the plan's schedule gives only the number of
 * sweeps.  Each sweep is a colour-class sweep with the chain's own draws (as
 * XZZX_ORDER_COLOUR) at its level's beta.  After sweep t the levels
 * (k, k + 1), k = t mod 2, t mod 2 + 2, ..., exchange their chains with
 * probability min(1, exp(delta (E_hi - E_lo))), delta the level spacing and
 * E_hi the energy of the chain at level k + 1: pair p = (k - t mod 2)/2
 * draws word p mod 4 of Philox(uid, 2^31 + 4b + P, t, p div 4), and the
 * exchange is accepted iff E_hi >= E_lo or u < T(E_lo - E_hi), where
 * T(n) = floor(prod over the set bits i of n of R_i / 2^32) in 64-bit fixed
 * point (the product starts at 2^64 - 1, each step keeps the high 64 bits),
 * R_0 = min(floor(2^64 exp(-delta 2^-16)), 2^64 - 1), R_{i+1} =
 * floor(R_i^2 / 2^64).  E_min, stop (phase 4t + k + 1) and the recovery are
 * as for colour sweeps.  EINVAL for another K or with the random-site order;
 * ERANGE if the ladder's tables and 64 chains do not fit in 64 KiB of LDS.
 * One chain per lane (XZZX_KERNEL_LADDER); the autotuner leaves the plan
 * unchanged and the serving loop rejects such plans. */
int xzzx_plan_set_ladder(xzzx_plan *plan, int levels, double beta_lo, double beta_hi);

/* Autotuner of the result-invariant knobs (kernel family, lanes per chain).
 * Builds a probe plan with the same lattice and weights and the first
 * probe_sweeps sweeps of the schedule, decodes n_syn random syndromes with
 * n_rep replicas once per candidate on `stream` (annealing stage timed with
 * HIP events, best of 3), and applies the fastest candidate to `plan`.
 * Candidates: the packed-row kernel where it applies, and the byte-state
 * kernel with 1, 2, 4, ..., 64 lanes per chain where its LDS fits.
 * times_ms[8] (may be NULL) receives the time of each candidate, index 0 for
 * the packed-row kernel and 1 + log2(lanes) for the byte-state kernel (-1 if
 * not tried).  Allocates and frees its own device buffers. */
typedef struct {
    int kernel;            /* chosen XZZX_KERNEL_ROWS or XZZX_KERNEL_BYTES */
    int lanes_per_chain;   /* chosen lanes (byte-state kernel) */
    float times_ms[8];
} xzzx_tune_result;
int xzzx_plan_autotune(xzzx_plan *plan, int n_rep, int n_syn, int probe_sweeps, void *stream,
                       xzzx_tune_result *out);

/* ---- device operations ---------------------------------------------------- */

/* Syndrome (Eq. (2)) of n configurations d_cfg[n][n_qubits] -> d_syn[n][n_stabs]. */
int xzzx_syndrome(const xzzx_plan *plan, const uint8_t *d_cfg, int64_t n, uint8_t *d_syn,
                  void *stream);

/* Greedy-matching references (Algs. 5-6): d_refs[n_syn][n_rep][n_qubits]
 * and their classes relative to replica 0, d_qcls[n_syn][n_rep].
 * mode: XZZX_GREEDY_RANDOM (Alg. 6), XZZX_GREEDY_SAME (Alg. 5),
 * XZZX_GREEDY_BOUNDARY (each defect to its nearest boundary). */
int xzzx_greedy_init(const xzzx_plan *plan, const uint8_t *d_syn, const uint32_t *d_uid,
                     int64_t n_syn, int n_rep, uint64_t greedy_seed, int mode, uint8_t *d_refs,
                     uint8_t *d_qcls, void *stream);

/* One group of syndromes sharing a plan.  Inputs: d_uid, and either d_syn
 * (decode) or d_refs + d_qcls (anneal only).  Required outputs: d_e_best,
 * d_cls, d_recovery.  Optional outputs (NULL to skip) hold per-coset minima,
 * the paper's output form R_0 L_P*, the best chain and per-chain results
 * (chain c of syndrome s at index s*4*n_rep + c). */
typedef struct {
    const xzzx_plan *plan;
    int64_t n_syn;
    int n_rep;
    const uint32_t *d_uid;       /* [n_syn] syndrome ids (RNG counters) */
    const uint8_t *d_syn;        /* [n_syn][n_stabs]; anneal: optional, checked against d_refs */
    uint8_t *d_refs;             /* [n_syn][n_rep][n_qubits]; decode writes it if non-NULL; anneal input */
    uint8_t *d_qcls;             /* [n_syn][n_rep] reference classes; written if non-NULL */
    int32_t *d_e_best;           /* [n_syn] min over cosets of E_P */
    uint8_t *d_cls;              /* [n_syn] P* */
    uint8_t *d_recovery;         /* [n_syn][n_qubits] minimum-energy configuration */
    uint8_t *d_paper_recovery;   /* [n_syn][n_qubits] R_0 L_P* (optional) */
    int32_t *d_e_cls;            /* [n_syn][4] E_P (optional) */
    int32_t *d_best_chain;       /* [n_syn] (optional) */
    int32_t *d_chain_emin;       /* [n_syn][4 n_rep] (optional) */
    int32_t *d_chain_stop;       /* [n_syn][4 n_rep] (optional) */
    int32_t *d_chain_e;          /* [n_syn][4 n_rep] final energies (optional) */
    uint8_t *d_chain_final;      /* [n_syn][4 n_rep][n_qubits] final states (optional) */
} xzzx_group;

/* Device workspace needed by xzzx_decode / xzzx_anneal for these groups. */
int xzzx_decode_workspace(const xzzx_group *groups, int n_groups, size_t *bytes);

/* Full decoder (Alg. 7) for every group: greedy init, annealing of all
 * chains of all groups in one persistent launch (uneven distances allowed),
 * per-syndrome reduction and recovery.  d_workspace: caller-owned device
 * memory of at least xzzx_decode_workspace() bytes.  ENOMEM if smaller. */
int xzzx_decode(const xzzx_group *groups, int n_groups, uint64_t greedy_seed,
                uint64_t anneal_seed, int greedy_mode, int flags, void *d_workspace,
                size_t workspace_bytes, void *stream);

/* As xzzx_decode, from caller-supplied references d_refs (no greedy
 * matching).  Its first stage (XZZX_FLAG_STAGE_GREEDY, included when no stage
 * is selected) takes the place of the greedy stage: it computes each
 * reference's class relative to replica 0 on the device (Alg. 7, Eqs.
 * (35)-(36); written to d_qcls if non-NULL) and, for groups whose d_syn is
 * non-NULL, checks that every reference has the group's syndrome (Alg. 7
 * requires boundary(C) = S), returning EINVAL if one does not.  That check
 * reads its result back, so it synchronizes `stream`; with d_syn set it is
 * refused (EINVAL) while `stream` is being captured.  Groups with d_syn NULL
 * are not checked and the call stays asynchronous. */
int xzzx_anneal(const xzzx_group *groups, int n_groups, uint64_t anneal_seed, int flags,
                void *d_workspace, size_t workspace_bytes, void *stream);

/* ---- decode without allocation -------------------------------------------- */

/* For callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid hipMalloc): xzzx_decode with the
 * workspace taken from a static device array of XZZX_NOALLOC_SCRATCH_BYTES
 * held by the library on each device it runs on, until the process ends.
 * The call allocates nothing: no device memory, and no stream or event (its
 * launches run in order on `stream`, so groups do not overlap each other).
 * The caller still allocates every group's inputs and outputs.  ERANGE if
 * xzzx_decode_workspace() for these groups exceeds the limit.  Every call on
 * one device shares that device's array, which keeps the last call's contents
 * (the decode clears what must start at zero itself): calls whose work
 * overlaps on one device -- on different streams or threads -- race and give
 * undefined results; serialise them.  Results equal xzzx_decode's. */
#define XZZX_NOALLOC_SCRATCH_BYTES (64u << 20)
int xzzx_decode_noalloc(const xzzx_group *groups, int n_groups, uint64_t greedy_seed,
                        uint64_t anneal_seed, int greedy_mode, int flags, void *stream);

/* ---- captured decode (hipGraph) -------------------------------------------- */

typedef struct xzzx_graph xzzx_graph;

/* Capture one xzzx_decode call (same arguments) into an executable HIP graph;
 * replaying it re-runs the decode on whatever the captured buffers hold. */
int xzzx_graph_create(const xzzx_group *groups, int n_groups, uint64_t greedy_seed,
                      uint64_t anneal_seed, int greedy_mode, int flags, void *d_workspace,
                      size_t workspace_bytes, void *stream, xzzx_graph **out);
int xzzx_graph_launch(xzzx_graph *graph, void *stream);
void xzzx_graph_destroy(xzzx_graph *graph);

/* ---- device limits (roofline peaks) ---------------------------------------- */

/* Microbenchmarks of the two limits the annealing kernels are measured
 * against, on the current device.  xzzx_probe_valu: int32 vector lane
 * operations per second of one instruction kind (0 v_xor_b32, 1 v_add_u32,
 * 2 v_bitop3_b32, 3 v_mad_u64_u32) issued by waves_per_simd (1..8) wavefronts
 * per SIMD on every CU, eight independent dependency chains per lane.
 * xzzx_probe_lds: LDS bytes read per second with conflict-free reads of
 * bytes_per_read (4, 8 or 16) bytes per lane.  iters (1..2^20) loop trips of
 * 128 operations (16 reads); best of 5 timed launches after a warm-up.  Each
 * call allocates and frees a small device buffer and synchronizes `stream`.
 * EINVAL for arguments out of range. */
int xzzx_probe_valu(int kind, int waves_per_simd, int iters, void *stream, double *lane_ops_per_s);
int xzzx_probe_lds(int bytes_per_read, int waves_per_simd, int iters, void *stream, double *bytes_per_s);

/* ---- serving loop (continuous batching) ------------------------------------ */

/* A server decodes single-syndrome requests as they arrive.  A scheduler
 * thread owns a HIP stream on the device current at creation and runs time
 * slices: at each slice boundary it admits queued requests (greedy references
 * computed on the device), advances every resident request by
 * sweeps_per_slice sweeps (more with many requests resident: see the
 * field) in one launch per kernel family (requests of
 * different distance and noise mix freely; a request advances a number of
 * sweeps inversely proportional to the sequential work of one of its sweeps,
 * so the tasks of a slice carry equal work), and finishes requests whose
 * schedule is complete (reduction and recovery on the device).  Chain states
 * stay in device memory between slices; counter-based random numbers make a
 * resumed chain identical to an uninterrupted one, so a request's result is
 * the same as from xzzx_decode with the same seeds, alone or in any mix.
 *
 * Admission: a request is admitted when a device slot is free (max_slots
 * slots of max_rep replicas on at most max_qubits qubits are allocated at
 * creation: the HBM budget) and the LDS its tasks need, summed over resident
 * requests, stays within lds_budget_bytes (0 = four times the device's total
 * LDS).  With a budget above the device's LDS a slice may hold more tasks
 * than run at once; the device starts queued tasks as earlier ones end, so
 * short tasks (small lattices) do not leave their waves idle.  A budget equal
 * to the device's LDS keeps every task of a slice running concurrently.
 *
 * Lanes per chain: each slice picks the largest power of two up to
 * max_lanes_per_chain for which the slice's wavefronts stay within max_waves
 * and its LDS within the budget; a request then runs on the byte-state kernel
 * with that many lanes per chain, or fewer where fewer already give each lane
 * one generator of a colour class (or, when the class has more generators
 * than that many lanes, at most one block of four), which cuts its latency
 * when the device is lightly loaded.  When even two lanes do not fit, every
 * request runs on its plan's own kernel choice.  Results do not depend on
 * this choice. */
typedef struct xzzx_server xzzx_server;

typedef struct {
    int max_slots;            /* resident requests (device slots) */
    int max_rep;              /* largest n_rep of a request */
    int max_qubits;           /* largest lattice (qubits) of a request */
    int sweeps_per_slice;     /* sweeps per slice of the largest resident lattice (>= 1) with up
                                 to 63 requests resident, one more sweeps_per_slice per further
                                 64; smaller lattices advance proportionally more */
    int max_pending;          /* queued requests before submit returns EAGAIN */
    int greedy_mode;          /* XZZX_GREEDY_* */
    int64_t lds_budget_bytes; /* 0: four times the device's total LDS */
    uint64_t greedy_seed;
    uint64_t anneal_seed;
    int max_lanes_per_chain;  /* 0: 64; 1: always the plan's own kernel; else a power of two <= 64 */
    int max_waves;            /* wavefronts per slice before lanes per chain shrink; 0: 32 per CU */
} xzzx_server_cfg;

typedef struct {
    const xzzx_plan *plan;    /* lattice, weights and schedule; must outlive the request */
    const uint8_t *syndrome;  /* host [n_stabs], copied by submit */
    uint32_t uid;             /* syndrome id (RNG counter) */
    int n_rep;
} xzzx_request;

typedef struct {
    int32_t e_best;           /* min over cosets of E_P */
    int32_t cls;              /* P*, relative to the replica-0 reference */
    int32_t e_cls[4];         /* E_P */
    uint8_t *recovery;        /* caller's host buffer [n_qubits] filled by poll (may be NULL) */
    double latency_s;         /* submit to result available on the host */
    double queue_s;           /* submit to admission */
} xzzx_result;

typedef struct {
    int64_t submitted, completed, rejected, slices;
    double p50_latency_s, p99_latency_s, mean_latency_s;
    double decodes_per_s;     /* completed requests over the busy interval */
    double attempts_per_s;    /* flip attempts of completed requests over the busy interval */
    double busy_s;            /* first admission to last completion */
} xzzx_serve_stats;

/* EINVAL for a bad configuration, ENOMEM if the slots do not fit. */
int xzzx_server_create(const xzzx_server_cfg *cfg, xzzx_server **out);

/* Queue a request; *ticket identifies it.  EAGAIN when max_pending requests
 * are queued, EINVAL if it does not fit the server's slots. */
int xzzx_server_submit(xzzx_server *srv, const xzzx_request *req, uint64_t *ticket);

/* Queue reqs[0..n-1] in order, as n calls of xzzx_server_submit would, with
 * one lock and one wake-up of the scheduler (callers feeding many requests
 * at once); tickets[i] (n entries, caller-owned) identifies request i.
 * Stops at the first request that fails (EINVAL as above; EAGAIN when the
 * queue fills) and returns its status; *n_done requests were queued. */
int xzzx_server_submit_many(xzzx_server *srv, const xzzx_request *reqs, int n, uint64_t *tickets, int *n_done);

/* XZZX_OK and the result (released by this call) if done; ENOTREADY while
 * queued or resident; EINVAL for an unknown or already collected ticket. */
int xzzx_server_poll(xzzx_server *srv, uint64_t ticket, xzzx_result *out);

/* Blocks until every submitted request has completed. */
int xzzx_server_drain(xzzx_server *srv);

/* Latency percentiles and throughput over the requests completed so far. */
int xzzx_server_stats(xzzx_server *srv, xzzx_serve_stats *out);

/* Finishes resident work, stops the scheduler and frees the device slots. */
void xzzx_server_destroy(xzzx_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* XZZX_SA_H */
