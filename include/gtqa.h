/*
 * gtqa.h — C ABI of the MI355X Trotter-step engine for the graph
 * tensor-network quantum annealer (GTQA) of arXiv:2409.12240.
 *
 * The library evolves a graph tensor network in the Vidal gauge
 * (Sec. II.A, Eq. vidal_gauge_tn) on a graph of maximum degree 3 under the
 * first-order Trotter circuit of a linear-schedule quantum anneal (App. F),
 * re-gauging with belief propagation (Sec. II.C, App. B Alg. 1, App. D
 * Alg. 2), and reads out single-qubit reduced density matrices, <Z>, the
 * rounded solution string and its objective (Sec. III.A).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Return codes: 0 = GTQA_OK; > 0 = warning (state still valid); < 0 = error.
 * Host arrays passed in are borrowed for the duration of the call only; the
 * library copies what it keeps.  Device memory is obtained through the
 * caller's allocator when one is given (gtqa_allocator), otherwise with
 * hipMalloc, and is released by the matching free call.  A state or pool is
 * bound to one HIP stream and must be used by one host thread at a time;
 * distinct states may be used concurrently.  Only the readout calls
 * synchronise with the stream; every other call only enqueues work, except
 * where BP convergence is tested (see gtqa_trotter_step) and where a call
 * says so.
 *
 * Indexing: vertices 0..n-1; edges given as [n_edges][2] int32 pairs with
 * u < v, sorted lexicographically, no repeats; an edge's id is its row.  The
 * legs of vertex a's tensor are its incident edges in ascending id order.
 * Physical index 0 is |0>, Z|0> = +|0>, and x_a = +1 stands for |0>
 * (Sec. III.A).
 */
#ifndef GTQA_H
#define GTQA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define GTQA_OK                 0
#define GTQA_WARN_BP_MAXITER    1   /* BP hit its sweep cap (App. B, K)      */
#define GTQA_WARN_JACOBI_CAP    2   /* a small SVD/eigen solve hit its cap   */
#define GTQA_ERR_ARG           -1   /* bad argument or option                */
#define GTQA_ERR_GRAPH         -2   /* degree 0 or > 3, self-loop, repeated
                                       or unsorted edge, improper colouring   */
#define GTQA_ERR_NOMEM         -3   /* allocation failed                     */
#define GTQA_ERR_HIP           -4   /* HIP runtime error                     */
#define GTQA_ERR_NUMERIC       -5   /* NaN/Inf in the inputs                 */
#define GTQA_ERR_STATE         -6   /* call not valid in the object's state  */
#define GTQA_BUSY              -7   /* pool admission: over the HBM budget   */
#define GTQA_ERR_UNSUPPORTED   -8   /* chi not built into this library       */

/* ---- options --------------------------------------------------------- */
#define GTQA_FP64       0   /* complex128 everywhere                          */
#define GTQA_MIXED      1   /* complex64 tensors, messages and BP arithmetic;
                               FP64 for the bond SVD (simple update) and for
                               the message factorisations of the gauge fix   */

#define GTQA_REGAUGE_EVERY_COLOUR 0   /* re-gauge after each colour class   */
#define GTQA_REGAUGE_EVERY_STEP   1   /* once per Trotter step, before U_X  */
#define GTQA_REGAUGE_NEVER        2
#define GTQA_REGAUGE_ADAPTIVE     3   /* after a colour class only where the
                                         Vidal residual R (App. C) of the
                                         instance exceeds residual_max: the
                                         occasional re-gauging of Sec. II.C */

#define GTQA_BP_COLOUR_ORDERED    0   /* Alg. 1 in place, edges by (colour, id) */
#define GTQA_BP_FLOODING          1   /* every message of a sweep from the previous
                                         sweep's messages (Jacobi order): the
                                         distance and stop rule of Alg. 1 unchanged */

typedef struct gtqa_allocator {
    void* (*alloc)(size_t bytes, void* ctx);   /* device memory, >= 256-B aligned */
    void  (*free)(void* ptr, void* ctx);
    void* ctx;
} gtqa_allocator;

typedef struct gtqa_instance {
    int32_t n;               /* vertices (qubits)                              */
    int32_t n_edges;
    const int32_t* edges;    /* [n_edges][2], u < v, lexicographically sorted  */
    const double* J;         /* [n_edges] couplings J_ab (Eq. objective_function) */
    const double* h;         /* [n] fields h_a                                  */
    const uint8_t* colour;   /* [n_edges] proper edge colouring, or NULL: the
                                library colours the edges (Misra-Gries)         */
} gtqa_instance;

typedef struct gtqa_options {
    int32_t chi;             /* bond-dimension cap (Alg. 3); built: 4, 8, 16    */
    int32_t precision;       /* GTQA_FP64 | GTQA_MIXED                          */
    double  bp_tol;          /* stop when dist/|E| < bp_tol (Alg. 1); <= 0 runs
                                exactly bp_max_sweeps sweeps                     */
    int32_t bp_max_sweeps;   /* K of Alg. 1                                     */
    double  svd_rel_cutoff;  /* singular values <= cutoff * sigma_0 are dropped */
    double  eig_rel_cutoff;  /* message pivots <= cutoff * max diag are dropped */
    int32_t regauge_policy;  /* GTQA_REGAUGE_*                                  */
    int32_t bp_schedule;     /* GTQA_BP_COLOUR_ORDERED | GTQA_BP_FLOODING        */
    void*   stream;          /* hipStream_t, NULL = default stream             */
    const gtqa_allocator* allocator;   /* NULL = hipMalloc/hipFree              */
    double  residual_max;    /* GTQA_REGAUGE_ADAPTIVE threshold on R; any finite
                                value (negative: always re-gauge)              */
    int32_t launch_mode;     /* GTQA_LAUNCH_DIRECT (default) | GTQA_LAUNCH_GRAPH */
} gtqa_options;

/* GTQA_LAUNCH_GRAPH: with re-gauging after every colour class and bp_tol > 0,
   each class's fixed launch sequence (simple update, phase flags, first BP
   sweep, stop-test reduction) and the gauge fix (Alg. 2 + gauge apply) are
   captured once per set of stepping instances as HIP graphs and replayed;
   the stop-test read-back, later sweeps, exact passes and compacted sweeps
   launch directly.  Results are identical to GTQA_LAUNCH_DIRECT.  Graphs
   are not used on the NULL stream, with step statistics or with stage
   timing on.  On ROCm 7 a graph replay costs more than the ~10 launches it
   replaces here, so direct launches are the default. */
#define GTQA_LAUNCH_DIRECT 0
#define GTQA_LAUNCH_GRAPH  1

/* Fills the defaults: chi 4, FP64, bp_tol 1e-10, 50 sweeps, svd cutoff 1e-12,
   eig cutoff 1e-14, re-gauge after every colour, colour-ordered BP,
   residual_max 1e-3, direct launches. */
void gtqa_default_options(gtqa_options* opt);

typedef struct gtqa_step_stats {
    int32_t n_regauges;          /* re-gaugings done in the step              */
    int32_t bp_sweeps[8];        /* BP sweeps of each re-gauging              */
    double  bp_dist[8];          /* final dist/|E| of each re-gauging (exact) */
    int32_t n_colours;
    double  log_fidelity;        /* sum over the step's two-qubit gates of
                                    log f, f = (sum_{k<chi} lambda_k^2)^2 on the
                                    normalised spectrum (Eq. gate_fidelity)    */
    double  max_trunc_error;     /* max over the step's gates of eps_ab^chi
                                    (Sec. II.C), normalised spectrum           */
    double  log_fidelity_total;  /* log F(M) since the state was created
                                    (Eq. total_fidelity)                      */
    double  residual[8];         /* GTQA_REGAUGE_ADAPTIVE: R after each colour
                                    class's gates, before the re-gauge decision
                                    (0 for classes the instance lacks)        */
    double  entropy;             /* S* after the step over the instance's
                                    bipartition (0 without one; see
                                    gtqa_set_bipartition)                     */
} gtqa_step_stats;

typedef struct gtqa_state gtqa_state;
typedef struct gtqa_pool gtqa_pool;

/* ---- single instance --------------------------------------------------- */

/* Builds |+>^N as a Vidal-gauge network with every bond of dimension 1
   (Sec. III.A) on a copy of the instance.  Validates the graph and the
   colouring (or computes one).  *out is set only on success. */
int gtqa_init_state(const gtqa_instance* inst, const gtqa_options* opt, gtqa_state** out);

/* One first-order Trotter step (App. F, Eq. discretizatoion): the interaction
   layer U_Z(theta_z) = prod_e exp(-i theta_z (J Z Z + h_a/D_a Z_a + h_b/D_b Z_b))
   applied by the simple update (App. E) with truncation to chi (Alg. 3),
   colour class by colour class in colour-id order, each class followed by
   re-gauging (Sec. II.C: symmetric gauge, BP from warm-start messages,
   Alg. 2) under the default policy; then the mixing layer
   U_X(theta_x) = prod_a exp(-i theta_x X_a) (Sec. II.D).  For the schedule
   s(t) = 1 - t/T with K = T/dt steps, step k takes theta_z = dt*k/K and
   theta_x = dt*(K-k)/K.  The BP stop test runs on the device after every
   sweep; the host reads its counters back once per batch of sweeps (as many
   as the quickest instance needed in the previous re-gauging, then one at a
   time), so with bp_tol > 0 the call synchronises once or a few times per
   colour class.  stats may be NULL. */
int gtqa_trotter_step(gtqa_state* st, double theta_z, double theta_x, gtqa_step_stats* stats);

/* The mixing layer U_X(theta_x) = prod_a exp(-i theta_x X_a) (Sec. II.D)
   alone, on every vertex of the network.  Single-site unitaries keep the
   Vidal gauge, so nothing is re-gauged.  Together with gtqa_trotter_step it
   composes other product formulas than the first-order one of App. F; the
   paper names higher-order formulas as the natural extension (Sec. VI).
   The symmetric second-order formula takes, for step k of K with midpoint
   s_k = (k - 1/2)/K, the interaction angle dt s_k and mixing half-angles
   a_k = dt (1 - s_k) / 2: one gtqa_x_layer(a_1) first, then
   gtqa_trotter_step(dt s_k, a_k + a_(k+1)) with a_(K+1) = 0.  The randomised
   first-order formula (random layer order per step, Sec. VI) applies the
   mixing layer of step k before its interaction layer on a coin: that
   mixing angle joins the previous step's (or a leading gtqa_x_layer).
   A non-finite theta_x returns GTQA_ERR_NUMERIC and changes nothing.
   Asynchronous on the state's stream. */
int gtqa_x_layer(gtqa_state* st, double theta_x);

/* Runs BP (Alg. 1) on the symmetric-gauge tensors T = Gamma lambda^(1/2)
   (Eq. symmetric_gauge) until dist/|E| < tol or max_sweeps sweeps (tol <= 0:
   exactly max_sweeps), in the state's bp_schedule: colour-ordered in place
   (edges by (colour, id)) or flooding.
   Start messages:
     GTQA_BP_WARM (default): diag(lambda)/sum(lambda), the warm start of
       Sec. II.C;
     GTQA_BP_RANDOM: Alg. 1's random initialisation m = A A^dagger /
       tr(A A^dagger) (App. B), a fresh d x d complex A per message (d the
       bond's dimension), entries uniform on the 2^-52 grid of [-1, 1):
       A[r][k] of direction dir (0: u->v, 1: v->u) of the instance's edge e
       takes outputs 2i (real part) and 2i + 1 (imaginary) of SplitMix64
       seeded with `seed` (Steele, Lea, Flood 2014; output j is the mix of
       seed + (j + 1) * 0x9E3779B97F4A7C15; value (x >> 11) * 2^-52 - 1),
       i = ((e * 2 + dir) * chi + r) * chi + k.  `seed` is ignored otherwise.
   With GTQA_BP_REGAUGE, Alg. 2 is applied to the converged messages.  The
   messages are kept for gtqa_readout(..., GTQA_READ_FROM_MESSAGES, ...).
   Returns GTQA_WARN_BP_MAXITER when tol > 0 and the sweep cap was reached
   first (the results are still written).  Unknown flag bits: GTQA_ERR_ARG.
   sweeps_out / dist_out (exact trace-norm dist/|E| of the last sweep) may be
   NULL.  Synchronises once per sweep when tol > 0 (the stop test). */
#define GTQA_BP_WARM     0u
#define GTQA_BP_REGAUGE  1u
#define GTQA_BP_RANDOM   2u
int gtqa_bp_converge(gtqa_state* st, double tol, int32_t max_sweeps, uint32_t flags, uint64_t seed,
                     int32_t* sweeps_out, double* dist_out);

/* Reads out rho_a (Eq. partial_dens), <Z_a> = rho00 - rho11, the rounded
   string x_a = +1 iff rho_a[0,0] > 1/2 (Eq. rounding_rule) and
   E(x) (Eq. objective_function, exact for couplings on a dyadic grid).
   FROM_VIDAL (default) uses rho ~ sum Gamma Gamma* prod lambda^2;
   FROM_MESSAGES uses T and the messages of the last gtqa_bp_converge.
   Outputs are host arrays, each may be NULL: z [n], rho [n][2][2][2]
   (re, im), x [n], energy [1].  Synchronises the stream. */
#define GTQA_READ_FROM_VIDAL     0u
#define GTQA_READ_FROM_MESSAGES  1u
int gtqa_readout(gtqa_state* st, uint32_t flags, double* z, double* rho, int8_t* x,
                 double* energy);

/* Vidal residual R (App. C) of the current network: the mean over the 2|E|
   edge directions a->b of the trace norm of 1_d - (d / tr M) M, where
   M[j][j'] = sum Gamma_a[.., j, ..] Gamma_a*[.., j', ..] prod_{c != b}
   lambda_ac^2 contracts every index of Gamma_a but the one on bond ab and
   d is that bond's dimension.  M is compared with the identity after
   division by its mean eigenvalue because the gauge fix leaves each Gamma_a
   a free positive scale.  R = 0 exactly in Vidal gauge.  Synchronises. */
int gtqa_vidal_residual(gtqa_state* st, double* R);

/* Mean-field entanglement entropy (Sec. III.C).  A bipartition side[n]
   (nonzero = subsystem A) marks the edges it cuts; S* = -sum over cut edges
   of sum_j lambda_j^2 log lambda_j^2 (Eqs. mean_field_schmidt,
   apprx_entropy; natural log) is then reported in gtqa_step_stats.entropy
   after every step and by gtqa_entropy on demand.  Copies side; synchronises. */
int gtqa_set_bipartition(gtqa_state* st, const uint8_t* side);
int gtqa_entropy(gtqa_state* st, double* S);

/* Host-only: the balanced bipartition of Eq. bipartition by spectral
   partitioning: vertices ordered by the Fiedler vector of the Laplacian
   L = D - Adj (sign: its largest-magnitude entry positive; ties by vertex
   id), and A = the prefix of that order minimising |dA| / (|A| |A-bar|)
   (the shortest on ties).  side_out [n] gets 1 for A; cut_out (may be NULL)
   the number of cut edges.  Needs no GPU. */
int gtqa_spectral_bipartition(int32_t n, int32_t n_edges, const int32_t* edges, uint8_t* side_out,
                              int32_t* cut_out);

/* BP-guided measurement sampling (Sec. IV.A, Eq. projection) of the whole
   string, for states whose marginals do not round (degenerate optima): the
   network is re-gauged (BP with tol / max_sweeps from the warm start, then
   Alg. 2); then for a = 0 .. n-1 in order, rho_a from the BP messages of the
   last re-gauging (Eq. partial_dens with Eq. bp_approx), x_a = +1 iff
   u[a] < rho_a[0][0] (u: the caller's uniforms in [0, 1)), Gamma_a projected
   on the outcome, and the network re-gauged again.  Outputs (host, each may
   be NULL): x [n], energy [1] = E(x), prob [n] = probability of each chosen
   outcome, sweeps [n] = BP sweeps of the re-gauging after each projection.
   The network ends in the measured product state.  n re-gaugings run in
   sequence; GTQA_WARN_BP_MAXITER if any hit max_sweeps. */
int gtqa_sample(gtqa_state* st, const double* u, double tol, int32_t max_sweeps, int8_t* x, double* energy,
                double* prob, int32_t* sweeps);

/* The network itself (Eq. vidal_gauge_tn), for checkpoint and resume and
   for starting from a given state.  gamma: host [n][2][chi][chi][chi]
   complex as (re, im) doubles, Gamma_a[i][j0][j1][j2] with legs in ascending
   incident-edge order, zero-padded beyond each bond's dimension (a missing
   leg of a vertex of degree < 3 uses index 0 only); lam: host [n_edges][chi]
   doubles, non-negative, non-increasing, lam[e][0] > 0, zero-padded (the
   bond dimension is the count of non-zero values).  In GTQA_MIXED the
   tensors are stored in complex64 (set rounds, get widens).  Set validates
   (non-finite: GTQA_ERR_NUMERIC; bad lambda: GTQA_ERR_ARG, nothing changed
   only if validation fails), copies and synchronises; it does not re-gauge.
   Get synchronises; either pointer may be NULL. */
int gtqa_set_network(gtqa_state* st, const double* gamma, const double* lam);
int gtqa_get_network(gtqa_state* st, double* gamma, double* lam);

void gtqa_free_state(gtqa_state* st);

/* The bond SVD of the simple update (App. E, Alg. 3) alone, for checking it:
   each of `count` caller-given 2chi x 2chi complex cores (host
   [count][2chi][2chi], row-major, (re, im) doubles) goes through the same
   device routine and launch layout as inside gtqa_trotter_step.  sigma
   [count][2chi] receives the column norms at exit in descending order, whose
   first chi are the Schmidt values the simple update keeps (before
   normalisation and the svd_rel_cutoff count); sweeps [count] the Jacobi
   sweeps used (more than 40: the cap was hit).  At chi = 4 the routine
   rotates only pairs touching the 4 largest columns and then checks that
   the discarded columns' total squared norm lies below the smallest kept
   squared norm (or below (svd_rel_cutoff sigma_0)^2), continuing on every
   pair otherwise, so the kept values are the chi largest.  Allocates device
   memory, runs on the NULL stream and synchronises.  Non-finite input:
   GTQA_ERR_NUMERIC. */
int gtqa_bond_svd(int32_t chi, int32_t count, const double* core, double svd_rel_cutoff, double* sigma,
                  int32_t* sweeps);

/* gtqa_bond_svd for callers that cannot allocate device memory (code under
   stream capture, tight serving loops, harnesses that forbid allocation):
   the same arguments, results and errors, but the device copies of the
   cores and results are staged in a library-owned static device array of
   2 MiB per device (held until the process ends) instead of allocated
   memory.  count may be at most gtqa_bond_svd_noalloc_max(chi) (1919 cores
   at chi = 4, 495 at chi = 8, 126 at chi = 16); more returns GTQA_ERR_ARG with a message on
   stderr.  All calls on one device share the array: calls that overlap on
   one device (other host threads) race and must be serialised by the
   caller.  Synchronous on the NULL stream. */
int gtqa_bond_svd_noalloc(int32_t chi, int32_t count, const double* core, double svd_rel_cutoff,
                          double* sigma, int32_t* sweeps);
int32_t gtqa_bond_svd_noalloc_max(int32_t chi);

/* Device bytes one instance needs (tensors, messages, gauge matrices, tables). */
size_t gtqa_footprint_bytes(int32_t n, int32_t n_edges, int32_t chi, int32_t precision);

const char* gtqa_strerror(int code);

/* Host-only: the library's Misra-Gries edge colouring (<= Delta+1 colours) of
   a sorted simple edge list; colour_out [n_edges].  Returns the number of
   colours or a negative error.  Needs no GPU. */
int gtqa_colour_edges(int32_t n, int32_t n_edges, const int32_t* edges, uint8_t* colour_out);

/* Library version string, for diagnostics. */
const char* gtqa_version(void);

/* ---- launch tuning (process-wide; set before pools capture or launch) --- */
/* Knobs the autotuner (paper_2409_12240_amd/autotune.py) picks by timing:
   SU_EDGES_PER_WAVE_CHI4: 2 or 4 edges of the chi=4 simple update per
     wavefront (32 or 16 lanes per edge; the Jacobi team's reduction order
     differs, so results differ at rounding level between the two);
   XCD_CONTIGUOUS: 0 or 1; with 1 the work-groups of the simple update, BP,
     Alg. 2, gauge-apply and residual-bound launches are reordered so each of
     the 8 XCDs takes a contiguous range of items (results unchanged);
   CANON_LANES_CHI4: 4 or 8 lanes per edge for Alg. 2 at chi=4 (one lane per
     column of the bond core, or an 8-lane team with two lanes per column;
     results differ at rounding level).
   Returns GTQA_ERR_ARG for an unknown knob or value.  Needs no GPU. */
#define GTQA_TUNE_SU_EDGES_PER_WAVE_CHI4 0
#define GTQA_TUNE_XCD_CONTIGUOUS         1
#define GTQA_TUNE_CANON_LANES_CHI4       2
int gtqa_set_tuning(int32_t knob, int32_t value);
int gtqa_get_tuning(int32_t knob, int32_t* value);

/* ---- batching and serving: a pool of instances sharing one chi/precision -- */

typedef struct gtqa_pool_options {
    gtqa_options base;        /* chi, precision, BP and cutoff options, stream */
    int64_t max_vertices;     /* capacity summed over resident instances       */
    int64_t max_edges;
    int32_t max_slots;
    int64_t budget_bytes;     /* admission budget (<= the capacity's footprint) */
} gtqa_pool_options;

int gtqa_pool_create(const gtqa_pool_options* opt, gtqa_pool** out);

/* Copies the instance into free capacity, initialises |+>^N and returns its
   slot.  GTQA_BUSY when its footprint does not fit the remaining budget or
   capacity (the pool is unchanged). */
int gtqa_pool_admit(gtqa_pool* pool, const gtqa_instance* inst, int32_t* slot_out);

/* One Trotter step (as gtqa_trotter_step) for `count` resident slots at once,
   slot slots[i] with its own angles; all listed slots advance together, each
   with its own BP stop decision.  stats may be NULL or [count]. */
int gtqa_pool_step(gtqa_pool* pool, const int32_t* slots, const double* theta_z,
                   const double* theta_x, int32_t count, gtqa_step_stats* stats);

/* As gtqa_readout for one slot.  Synchronises the pool's stream. */
int gtqa_pool_readout(gtqa_pool* pool, int32_t slot, double* z, double* rho, int8_t* x,
                      double* energy);

/* Frees the slot's capacity for later admissions. */
int gtqa_pool_release(gtqa_pool* pool, int32_t slot);

/* Bytes of the budget still free; resident slot count. */
int64_t gtqa_pool_free_bytes(const gtqa_pool* pool);
int32_t gtqa_pool_resident(const gtqa_pool* pool);

void gtqa_pool_free(gtqa_pool* pool);

/* As gtqa_sample for `count` resident slots at once (their qubit a is
   measured in the same launches); u, x, prob and sweeps concatenate the
   slots' vertices in the order of slots[], energy is [count]. */
int gtqa_pool_sample(gtqa_pool* pool, const int32_t* slots, int32_t count, const double* u, double tol,
                     int32_t max_sweeps, int8_t* x, double* energy, double* prob, int32_t* sweeps);

/* Changes the BP stop rule (Alg. 1: dist/|E| < tol, at most max_sweeps
   sweeps; tol <= 0 runs exactly max_sweeps) for the pool's later steps.
   GTQA_ERR_ARG for a non-finite tol or max_sweeps < 1. */
int gtqa_pool_set_bp(gtqa_pool* pool, double tol, int32_t max_sweeps);

/* As gtqa_set_network / gtqa_get_network for one resident slot. */
int gtqa_pool_set_network(gtqa_pool* pool, int32_t slot, const double* gamma, const double* lam);
int gtqa_pool_get_network(gtqa_pool* pool, int32_t slot, double* gamma, double* lam);

/* As gtqa_set_bipartition / gtqa_entropy for one resident slot. */
int gtqa_pool_set_bipartition(gtqa_pool* pool, int32_t slot, const uint8_t* side);
int gtqa_pool_entropy(gtqa_pool* pool, int32_t slot, double* S);

/* As gtqa_x_layer for `count` distinct resident slots, theta_x [count] one
   angle per slot (host array). */
int gtqa_pool_x_layer(gtqa_pool* pool, const int32_t* slots, int32_t count, const double* theta_x);

/* As gtqa_vidal_residual for `count` resident slots at once; R [count]. */
int gtqa_pool_residual(gtqa_pool* pool, const int32_t* slots, int32_t count, double* R);

/* Cumulative BP sweeps and re-gaugings of a slot since its admission (the
   sweeps of Alg. 1 summed over re-gaugings).  Synchronises the stream. */
int gtqa_pool_bp_totals(gtqa_pool* pool, int32_t slot, int64_t* sweeps, int64_t* regauges);

/* ---- stage timing (measurement) --------------------------------------- */
/* When enabled, every kernel launch of a pool is bracketed by HIP events on
   the pool's stream; reading sums the elapsed times per stage.  Enabling
   clears earlier records.  Reading synchronises the stream.  items counts
   the work items (edges or vertices) the stage's launches covered. */
#define GTQA_STAGE_SIMPLE_UPDATE 0
#define GTQA_STAGE_BP_INIT       1
#define GTQA_STAGE_BP_SWEEP      2
#define GTQA_STAGE_BP_REDUCE     3
#define GTQA_STAGE_CANONICALISE  4
#define GTQA_STAGE_GAUGE_APPLY   5
#define GTQA_STAGE_X_LAYER       6
#define GTQA_STAGE_READOUT       7
#define GTQA_STAGE_RESIDUAL      8
#define GTQA_N_STAGES            9
int gtqa_pool_profile(gtqa_pool* pool, int32_t enable);
/* As gtqa_pool_profile, for the stages whose bit is set in stage_mask
   (bit GTQA_STAGE_x); the other stages launch without events, so timing one
   stage costs the others nothing.  gtqa_pool_profile(pool, e) is
   gtqa_pool_profile_stages(pool, e ? all stages : 0).  Bits at or above
   GTQA_N_STAGES return GTQA_ERR_ARG. */
int gtqa_pool_profile_stages(gtqa_pool* pool, uint32_t stage_mask);
int gtqa_pool_profile_read(gtqa_pool* pool, int32_t stage, int64_t* launches, double* total_ms,
                           int64_t* items);
/* Time the launches of one gtqa_pool_step (or gtqa_trotter_step) call in
   every `every` (the first after this call or after enabling, then every
   every-th); launches outside steps are always timed.  The events cost the
   step a few per cent, so sampling keeps the timed steps' rate close to the
   unmeasured one.  Default 1 (every step); every < 1 returns GTQA_ERR_ARG.
   Does not synchronise or clear records. */
int gtqa_pool_profile_sample(gtqa_pool* pool, int32_t every);

#ifdef __cplusplus
}
#endif
#endif /* GTQA_H */
