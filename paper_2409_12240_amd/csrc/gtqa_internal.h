// Internal layout of a GTQA pool in device memory and the kernel launchers.
//
// Every resident instance ("slot") owns a contiguous range of vertices and
// edges in pool-wide arrays, so one kernel launch can cover the items of
// many instances.  Layout (chi fixed per pool, S = double or float):
//   gam  [V][2][chi][chi][chi]  complex<S>  Gamma_a[i][j0][j1][j2], legs in
//                                           ascending incident-edge order;
//                                           missing legs (degree < 3) carry
//                                           index 0 only
//   lam  [E][chi]               double      lambda_e, descending, zero-padded
//   msg  [E][2][chi][chi]       complex<S>  m_{u->v}, m_{v->u} (u < v)
//   xg   [E][2][chi][chi]       complex<S>  gauge maps of the last
//                                           canonicalisation, sqrt(lambda_old)
//                                           folded in (computed in FP64, stored
//                                           in the precision they are applied in)
//   vedge[V][3] int32 incident edge per leg (-1 = missing leg)
//   eend [E][2] int32 endpoints; eleg [E][2] int32 leg position at u, v
//   vmeta[V] int4 {gauge-map index of leg 0, 1, 2 (2*edge + side, -1 = missing),
//                  slot}
//   bpmeta[E][2] int4 per direction d (message leaving endpoint d):
//                {vertex, incoming message index on the first other leg,
//                 on the second other leg (2*edge + direction, -1 = missing),
//                 leg | colour of the first << 8 | colour of the second << 16}
// Missing legs behave as bonds of dimension 1 with lambda = (1, 0, ...)
// and message e0 e0^T.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gtqa {

struct DevPool {
    void* gam;
    double* lam;
    void* msg;
    void* xg;              // complex<S> gauge maps
    const int32_t* vedge;
    const int32_t* eend;
    const int32_t* eleg;
    const int4* bpmeta;
    const int4* vmeta;
    int xcd_remap;         // work-group order remapped so each XCD takes a contiguous item range
    const double* J;
    const double* hD;      // h_a / D_a
    const double* h;       // h_a
    const int32_t* eslot;
    const int32_t* vslot;
    double* edist;         // per-edge upper bound on the BP distance of the last sweep
    double* edlo;          // per-edge lower bound (Frobenius norms)
    double* edexact;       // per-edge exact trace-norm distance (when computed)
    void* mold;            // [E][2][chi][chi] complex<S>: the messages the last sweep replaced
    const uint8_t* ecol;   // [E] colour class of each edge
    double* rho;           // [V][2][2] complex<double> readout
    double* zval;          // [V] <Z_a>
    // per-slot
    const double* theta;   // [slots][2]: theta_z, theta_x
    int32_t* sflag;        // FLAG_* bits of the current phase
    const int32_t* smask;  // bit c: colour class c of the slot is non-empty
    int32_t* ssweeps;      // BP sweeps done in the current re-gauging
    double* sdist;         // dist/|E| after the last sweep
    const int32_t* s_e0;
    const int32_t* s_ne;
    const int32_t* s_v0;
    const int32_t* s_nv;
    int32_t* swarn;        // warning bits per slot (Jacobi cap)
    int64_t* stot;         // [slots][2] cumulative BP sweeps, re-gaugings since admission
    double* elogf;         // [E] log of the gate fidelity estimate of the edge's last simple update
    double* eeps;          // [E] truncation error eps of the edge's last simple update
    int32_t* efix;         // [E] 1: the last simple update's restricted bond SVD failed the
                           //     kept-set check and the edge waits for the every-pair redo
    double* sfid;          // [slots][3]: step sum log f, step max eps, cumulative sum log f
    const uint8_t* ecut;   // [E] 1 if the instance's bipartition cuts the edge
    double* sent;          // [slots] mean-field entanglement entropy S* over the cut edges
    double* vres;          // [V] sum over the vertex's legs of the local-orthogonality residual
                           //     (or of its lower bound ||D||_F in the bounds pass)
    double* vres_hi;       // [V] upper bound sum_legs min(sqrt(d) ||D||_F, sum |D_ij|)
    double* sres;          // [slots] Vidal residual R of the slot (last computed; lower bound
                           //         after a bounds pass)
    double* sres_hi;       // [slots] upper bound on R after a bounds pass (= sres when exact)
    double res_max;        // adaptive re-gauging threshold on R
    double* senergy;       // E(x) per slot
    int8_t* xbits;         // [V] rounded string
    double svd_cut;
    double eig_cut;
    double bp_tol;
    int bp_flood;          // 1: flooding BP schedule (every message of a sweep from the
                           //    previous sweep's, read from mold), 0: colour-ordered in place
    double* su_ws;         // chi >= 16: simple-update workspace (QR data, R factors, kept
                           //            vectors) for su_chunk edges at a time
    int su_chunk;
    // null, or the BP stop-test counters [0] sweeping, [1] undecided: the
    // canonicalisation and gauge kernels then return at once unless both are
    // zero (Alg. 2 enqueued ahead of the host's read of the stop test)
    const int32_t* tail_gate;
};

enum : int32_t { FLAG_ACTIVE = 1, FLAG_BP_DONE = 2, FLAG_APPLY_X = 4, FLAG_UNDECIDED = 8, FLAG_BP_CAPPED = 16 };
enum : int32_t { WARN_JACOBI = 1 };
// BP stop-test counter [3] holds kSweepBias - (fewest sweeps a converged slot needed)
constexpr int32_t kSweepBias = 1 << 20;

// launchers (defined in gtqa_kernels.hip); items are device index lists
int launch_init_plus(int chi, int prec, const DevPool& p, const int32_t* verts, int nv,
                     const int32_t* edges, int ne, hipStream_t s);
int launch_simple_update(int chi, int prec, const DevPool& p, const int32_t* edges, int ne,
                         hipStream_t s);
int launch_warm_messages(int chi, int prec, const DevPool& p, const int32_t* edges, int ne,
                         hipStream_t s);
// One colour class `cls` of a BP sweep over the work records `recs` (three
// int4 per edge, from launch_bp_records).  In the first sweep of a
// re-gauging the messages not yet updated (edges of later classes, and the
// edge's own old messages) are the warm-start messages diag(lambda)/sum(lambda).
// gate (may be null): a device count of slots still sweeping; 0 skips the launch.
int launch_bp_sweep_class(int chi, int prec, const DevPool& p, const int4* recs, int ne,
                          int first_sweep, int cls, const int32_t* gate, hipStream_t s);
// Flooding schedule: copy the listed edges' messages to mold (the previous
// iterate every message of the next sweep is computed from) for the slots
// still sweeping; launched for every class before the sweep's class kernels.
int launch_bp_snapshot(int chi, int prec, const DevPool& p, const int4* recs, int ne, hipStream_t s);
// Work records of `n` listed edges: out[3i], out[3i+1] = the direction
// records of edge items[i], out[3i+2] = (edge, slot, 0, 0).
int launch_bp_records(const DevPool& p, const int32_t* items, int n, int4* out, hipStream_t s);
// counters[0] += slots still sweeping, counters[1] += slots whose bounds do
// not decide the stop test (they pause until the exact pass), counters[2] +=
// slots stopped at max_sweeps unconverged; force_exact marks every active
// slot undecided.
int launch_bp_reduce(const DevPool& p, const int32_t* slots, int nslots, int32_t* counters,
                     int force_exact, int max_sweeps, hipStream_t s);
// force: every active slot (an exact distance for reporting), otherwise
// only the undecided ones
int launch_bp_exact(int chi, int prec, const DevPool& p, const int32_t* edges, int ne, int force, hipStream_t s);
int launch_bp_reduce_exact(const DevPool& p, const int32_t* slots, int nslots, int32_t* counters,
                           int force, int max_sweeps, hipStream_t s);
int launch_canonicalise(int chi, int prec, const DevPool& p, const int32_t* edges, int ne,
                        hipStream_t s);
int launch_gauge_apply(int chi, int prec, const DevPool& p, const int32_t* verts, int nv,
                       int apply_x, hipStream_t s);
int launch_x_layer(int chi, int prec, const DevPool& p, const int32_t* verts, int nv,
                   hipStream_t s);
int launch_readout(int chi, int prec, const DevPool& p, const int32_t* verts, int nv,
                   int from_messages, hipStream_t s);
int launch_energy(const DevPool& p, const int32_t* slots, int nslots, hipStream_t s);
// phase < 0: every slot active with U_X fused (re-gauge once per step);
// otherwise slot active iff its colour class `phase` is non-empty, with U_X
// fused iff `phase` is its last non-empty class.  Resets sweep counters;
// clear4 (may be null): four int32 counters also set to zero.
int launch_phase_flags(const DevPool& p, const int32_t* slots, int nslots, int phase,
                       hipStream_t s, int32_t* clear4 = nullptr);

// Compaction of the per-class edge lists to the slots still running BP.
// seg: [ncol][nslots][2] (offset within the class list, length) of each
// plan slot's edges; full: the class lists; out: compacted lists at the same
// class offsets (full_rec, out_rec: their work records, three per position);
// counts[c] = compacted length of class c.
int launch_bp_compact(const DevPool& p, const int32_t* slots, int nslots, int ncol, const int32_t* seg,
                      const int64_t* cls_off, const int32_t* full, int32_t* out, const int4* full_rec,
                      int4* out_rec, int32_t* counts, int32_t* scratch, hipStream_t s);

// Vidal residual R (App. C) of every listed slot into p.sres (= p.sres_hi).
// mode RES_EXACT: all listed slots; RES_BOUNDS: lower/upper bounds from the
// Frobenius and entrywise norms (no SVD) into sres / sres_hi (at chi = 16 the
// exact value as both); RES_UNDECIDED: exact, only for slots flagged
// FLAG_UNDECIDED.
enum { RES_EXACT = 0, RES_BOUNDS = 1, RES_UNDECIDED = 2 };
int launch_residual(int chi, int prec, const DevPool& p, const int32_t* verts, int nv, const int32_t* slots,
                    int nslots, int mode, hipStream_t s);
// adaptive phase: slot active iff its class `phase` is non-empty and R > res_max, decided from
// sres / sres_hi; slots the bounds do not decide get FLAG_UNDECIDED.  counters[0] += active,
// counters[1] += undecided (the caller zeroes them).  Never fuses U_X.
int launch_phase_flags_adaptive(const DevPool& p, const int32_t* slots, int nslots, int phase, int32_t* counters,
                                hipStream_t s);
// second stage for FLAG_UNDECIDED slots once their exact R is in sres: counters[0] += active
int launch_phase_flags_adaptive_final(const DevPool& p, const int32_t* slots, int nslots, int32_t* counters,
                                      hipStream_t s);

// per-slot sum of log f and max eps over the slot's edges (one simple update
// each per step); adds the sum to the slot's cumulative log-fidelity
int launch_fidelity_reduce(const DevPool& p, const int32_t* slots, int nslots, int chi, hipStream_t s);

// Process-wide launch configuration, chosen by the autotuner (set before
// pools capture or launch): edges per wavefront of the chi=4 simple update
// (2 or 4), the XCD-contiguous work-group order (0 or 1) and the lanes per
// edge of Alg. 2 at chi=4 (4 or 8).
struct Tuning {
    int su_epw_chi4;
    int xcd_remap;
    int canon_lanes_chi4;  // Alg. 2 at chi = 4: 4 (one lane per core column) or 8 lanes per edge
};
Tuning& tuning();

// S* (Sec. III.C, Eq. apprx_entropy) of the listed slots into p.sent
int launch_entropy(const DevPool& p, const int32_t* slots, int nslots, int chi, hipStream_t s);

// BP-guided sampling (Sec. IV.A), qubit `a` of every listed slot that has
// it: x = +1 iff u[i] < rho[v][0][0] (rho from the last readout of v =
// s_v0 + a), xbits[v] = x, prob[i] = probability of x, Gamma_v projected on
// the outcome (Eq. projection).  Flags: slots with qubit `a` active.
int launch_sample_project(int chi, int prec, const DevPool& p, const int32_t* slots, int nslots, int a,
                          const double* u, double* prob, hipStream_t s);
int launch_sample_flags(const DevPool& p, const int32_t* slots, int nslots, int a, hipStream_t s);

// x[0 .. n) = 0 by a kernel (safe inside captured graphs, unlike a memset node)
int launch_zero_i32(int32_t* x, int n, hipStream_t s);

// The simple update's bond SVD alone on `count` caller-given 2chi x 2chi
// cores (device, [count][2chi][2chi] complex as re, im): sigma [count][2chi]
// column norms at exit, descending; sweeps [count].
int launch_core_svd(int chi, const double* core, int count, double cut, double* sigma, int32_t* sweeps,
                    hipStream_t s);

// Alg. 1's random start m = A A^dagger / tr (App. B) for the listed edges'
// messages, A's entries from SplitMix64 outputs addressed by the instance's
// edge id, direction and entry (see the kernel).
int launch_random_messages(int chi, int prec, const DevPool& p, const int32_t* edges, int ne, uint64_t seed,
                           hipStream_t s);

bool chi_supported(int chi);

// chi = 16 (gtqa_wide.hip): simple update in su_chunk-edge chunks through
// p.su_ws (three kernels per chunk), the BP class sweep, Alg. 2 and the gauge
// application with the same contracts as the launchers above.
size_t su_ws_bytes_per_edge(int chi);
int launch_wide_simple_update(int chi, int prec, const DevPool& p, const int32_t* edges, int ne, hipStream_t s);
int launch_wide_bp_sweep_class(int chi, int prec, const DevPool& p, const int4* recs, int ne, int first_sweep,
                               int cls, const int32_t* gate, hipStream_t s);
int launch_wide_canonicalise(int chi, int prec, const DevPool& p, const int32_t* edges, int ne, hipStream_t s);
int launch_wide_residual(int chi, int prec, const DevPool& p, const int32_t* verts, int nv, int mode,
                         hipStream_t s);
int launch_wide_gauge_apply(int chi, int prec, const DevPool& p, const int32_t* verts, int nv, int apply_x,
                            hipStream_t s);

}  // namespace gtqa
