// Host side of the GTQA engine: the C ABI of include/gtqa.h, pools of
// resident instances, instance validation and the library's edge colouring.
//
// A single-instance state is a pool with one slot.  A pool owns, for a fixed
// chi and precision, device arrays sized for its capacity; admitted
// instances take contiguous vertex and edge ranges.  A Trotter step over a
// set of slots enqueues one launch per kernel stage covering every item of
// every listed slot.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "gtqa.h"
#include "gtqa_internal.h"

using gtqa::DevPool;

namespace {

constexpr int kMaxColours = 8;   // Delta + 1 <= 4 for degree <= 3
constexpr int64_t kSuChunk = 8192; // chi >= 16: edges per simple-update chunk (about 0.3 MB of workspace each)

// ------------------------------------------------------------------ colouring
// Misra-Gries constructive Vizing colouring with the tie-breaks:
//  * edges in id order; for (u, v), u < v, the fan is built at u from v;
//  * the fan grows by the first neighbour of u (ascending id) not yet in it
//    whose edge to u carries a colour free at the current last fan vertex;
//  * c = lowest colour free at u, d = lowest free at the last fan vertex;
//  * the path from u alternating d, c, d, ... has its two colours swapped;
//  * w = first fan vertex (fan order) whose prefix is still a fan and at which
//    d is free; that prefix is rotated and (u, w) gets d.
class MisraGries {
  public:
    MisraGries(int n, int m, const int32_t* edges) : n_(n), m_(m), ed_(edges) {
        nbr_.assign(n, {});
        for (int e = 0; e < m; ++e) {
            nbr_[ed_[2 * e]].push_back({ed_[2 * e + 1], e});
            nbr_[ed_[2 * e + 1]].push_back({ed_[2 * e], e});
        }
        int delta = 0;
        for (int a = 0; a < n; ++a) {
            std::sort(nbr_[a].begin(), nbr_[a].end());
            delta = std::max<int>(delta, (int)nbr_[a].size());
        }
        nc_ = delta + 1;
        col_.assign(m, -1);
        slot_.assign((size_t)n * nc_, -1);
    }

    int run(uint8_t* out) {
        for (int e0 = 0; e0 < m_; ++e0) {
            const int u = ed_[2 * e0], v = ed_[2 * e0 + 1];
            std::vector<int> fan{v};
            for (;;) {
                const int last = fan.back();
                int next = -1;
                for (const auto& nb : nbr_[u]) {
                    if (std::find(fan.begin(), fan.end(), nb.first) != fan.end()) continue;
                    const int c = col_[nb.second];
                    if (c >= 0 && free_at(last, c)) { next = nb.first; break; }
                }
                if (next < 0) break;
                fan.push_back(next);
            }
            const int c = lowest_free(u), d = lowest_free(fan.back());
            if (c < 0 || d < 0) return -1;
            if (c != d) {
                std::vector<int> path;
                int x = u, want = d;
                for (;;) {
                    const int e = slot_[(size_t)x * nc_ + want];
                    if (e < 0) break;
                    path.push_back(e);
                    x = other(e, x);
                    want = (want == d) ? c : d;
                }
                for (int e : path) set(e, -1);
                for (size_t i = 0; i < path.size(); ++i) set(path[i], (i % 2 == 0) ? c : d);
            }
            int k = -1;
            for (size_t i = 0; i < fan.size(); ++i) {
                if (i > 0) {
                    const int ce = col_[edge_of(u, fan[i])];
                    if (ce < 0 || !free_at(fan[i - 1], ce)) break;
                }
                if (free_at(fan[i], d)) { k = (int)i; break; }
            }
            if (k < 0) return -1;
            for (int i = 0; i < k; ++i) {
                const int ei = edge_of(u, fan[i]);
                const int en = edge_of(u, fan[i + 1]);
                const int cn = col_[en];
                set(en, -1);
                set(ei, cn);
            }
            set(edge_of(u, fan[k]), d);
        }
        int used = 0;
        for (int e = 0; e < m_; ++e) {
            out[e] = (uint8_t)col_[e];
            used = std::max(used, col_[e] + 1);
        }
        return used;
    }

  private:
    bool free_at(int x, int c) const { return slot_[(size_t)x * nc_ + c] < 0; }
    int lowest_free(int x) const {
        for (int c = 0; c < nc_; ++c)
            if (free_at(x, c)) return c;
        return -1;
    }
    int other(int e, int x) const { return ed_[2 * e] == x ? ed_[2 * e + 1] : ed_[2 * e]; }
    int edge_of(int x, int y) const {
        for (const auto& nb : nbr_[x])
            if (nb.first == y) return nb.second;
        return -1;
    }
    void set(int e, int c) {
        const int a = ed_[2 * e], b = ed_[2 * e + 1];
        const int old = col_[e];
        if (old >= 0) {
            slot_[(size_t)a * nc_ + old] = -1;
            slot_[(size_t)b * nc_ + old] = -1;
        }
        col_[e] = c;
        if (c >= 0) {
            slot_[(size_t)a * nc_ + c] = e;
            slot_[(size_t)b * nc_ + c] = e;
        }
    }
    int n_, m_, nc_ = 1;
    const int32_t* ed_;
    std::vector<std::vector<std::pair<int, int>>> nbr_;
    std::vector<int> col_;
    std::vector<int> slot_;
};

// ------------------------------------------------------------------ ranges
struct RangeAlloc {
    std::vector<std::pair<int64_t, int64_t>> free_;   // (start, length), sorted
    void reset(int64_t cap) { free_.assign(1, {0, cap}); }
    int64_t take(int64_t len) {
        if (len == 0) return 0;
        for (size_t i = 0; i < free_.size(); ++i) {
            if (free_[i].second >= len) {
                const int64_t s = free_[i].first;
                free_[i].first += len;
                free_[i].second -= len;
                if (free_[i].second == 0) free_.erase(free_.begin() + i);
                return s;
            }
        }
        return -1;
    }
    void give(int64_t s, int64_t len) {
        if (len == 0) return;
        free_.push_back({s, len});
        std::sort(free_.begin(), free_.end());
        std::vector<std::pair<int64_t, int64_t>> merged;
        for (const auto& r : free_) {
            if (!merged.empty() && merged.back().first + merged.back().second == r.first)
                merged.back().second += r.second;
            else
                merged.push_back(r);
        }
        free_.swap(merged);
    }
};

struct SlotInfo {
    bool used = false;
    int64_t v0 = 0, nv = 0, e0 = 0, ne = 0;
    int ncol = 0;
    int mask = 0;
    size_t bytes = 0;
    std::vector<std::vector<int32_t>> cls;   // global edge ids per colour
    std::vector<int32_t> edges;              // the instance's edge list (local ids), for bipartitions
};

size_t complex_bytes(int precision) { return precision == GTQA_MIXED ? 8 : 16; }

size_t vertex_bytes(int chi, int precision) {
    return (size_t)2 * chi * chi * chi * complex_bytes(precision)  // Gamma
           + 3 * 4 + 8 + 8 + 4                                      // vedge, hD, h, vslot
           + 64 + 8 + 1                                             // rho, z, x
           + 16                                                     // residual terms and bounds
           + 16                                                     // gauge-apply metadata
           + 8;                                                     // vertex work lists
}

size_t edge_bytes(int chi, int precision) {
    return (size_t)chi * 8                                          // lambda
           + (size_t)2 * chi * chi * complex_bytes(precision)       // messages
           + (size_t)2 * chi * chi * complex_bytes(precision)       // gauge maps
           + (size_t)2 * chi * chi * complex_bytes(precision)       // messages the last BP sweep replaced
           + 8 + 8 + 8 + 4 + 1                                      // eend, eleg, J, eslot, colour
           + 32                                                     // BP direction metadata
           + 8 + 8 + 8                                              // distance, bound, exact
           + 8 + 8 + 4                                              // log f, eps, redo flag
           + 1                                                      // cut by the bipartition
           + 20                                                     // edge work lists
           + 96;                                                    // BP work records (plan, compacted)
}

}  // namespace

struct gtqa_pool {
    int chi = 4, prec = 0;
    gtqa_options opt{};
    gtqa_allocator alloc{};
    bool has_alloc = false;
    hipStream_t stream = nullptr;
    int64_t maxV = 0, maxE = 0;
    int maxS = 0;
    int64_t budget = 0, used_bytes = 0;
    std::vector<void*> blocks;
    DevPool dp{};
    // device
    void* gam = nullptr;
    double* lam = nullptr;
    void* msg = nullptr;
    void* xg = nullptr;
    int32_t *vedge = nullptr, *eend = nullptr, *eleg = nullptr, *eslot = nullptr, *vslot = nullptr;
    int4* bpmeta = nullptr;
    int4* vmeta = nullptr;
    double *J = nullptr, *hD = nullptr, *h = nullptr, *edist = nullptr, *rho = nullptr, *zval = nullptr;
    double *edlo = nullptr, *edexact = nullptr;
    void* mold = nullptr;
    uint8_t* ecol = nullptr;
    int8_t* xbits = nullptr;
    double* theta = nullptr;
    int32_t *sflag = nullptr, *smask = nullptr, *ssweeps = nullptr, *swarn = nullptr;
    int64_t* stot = nullptr;
    double *elogf = nullptr, *eeps = nullptr, *sfid = nullptr;
    int32_t* efix = nullptr;
    double *vres = nullptr, *sres = nullptr, *vres_hi = nullptr, *sres_hi = nullptr;
    uint8_t* ecut = nullptr;
    double* sent = nullptr;
    double* sbuf = nullptr;         // [2][slots] sampling: uniforms in, probabilities out
    double *sdist = nullptr, *senergy = nullptr;
    int32_t *s_e0 = nullptr, *s_ne = nullptr, *s_v0 = nullptr, *s_nv = nullptr;
    int32_t* lists = nullptr;       // work lists
    int32_t* clists = nullptr;      // compacted class lists (same offsets as the class lists)
    int4* crec = nullptr;           // BP work records of the class lists (3 per position)
    int4* ccrec = nullptr;          // ... and of the compacted class lists
    int32_t* seg = nullptr;         // [ncol][nslots][2] per-slot class segments of the plan
    int64_t* d_cls_off = nullptr;   // class offsets
    int32_t* cscratch = nullptr;    // [ncol][nslots] compacted offsets
    int32_t* d_counts = nullptr;    // [ncol] compacted class lengths
    double* su_ws = nullptr;        // chi >= 16: simple-update workspace for su_chunk edges
    int su_chunk = 0;
    int32_t* h_counts = nullptr;    // pinned mirror
    int32_t* d_notdone = nullptr;   // [0] slots sweeping, [1] undecided, [2] capped; [4..5] adaptive
    int32_t* h_notdone = nullptr;   // pinned: [0..1] counters, [2..2+kMaxColours) class counts,
                                    // [2+kMaxColours..+2) adaptive counters, [4+kMaxColours] capped
    int spec_rounds = 1;            // BP sweeps the last re-gauging took: enqueued per read-back
    bool tail_spec = true;          // the last re-gauging's BP stopped at its first read-back:
                                    // enqueue Alg. 2 gated ahead of the next one's
    hipEvent_t ev_rb = nullptr;     // marks the stop-test copy, so the host waits for it alone
    // host
    std::vector<SlotInfo> slots;
    RangeAlloc vr, er;
    std::vector<double> h_theta;
    // cached plan
    std::vector<int32_t> plan_key;
    int64_t off_cls[kMaxColours + 1] = {0};
    int64_t off_alle = 0, off_allv = 0, off_slots = 0;
    int64_t n_alle = 0, n_allv = 0;
    int plan_ncol = 0;
    int resident = 0;
    // captured launch sequences (GTQA_LAUNCH_GRAPH), valid for plan_key == graph_key
    std::vector<int32_t> graph_key;
    bool graphs_ok = false;
    hipGraphExec_t g_head[kMaxColours] = {};
    hipGraphExec_t g_sweep = nullptr;
    hipGraphExec_t g_tail = nullptr;
    bool graphs_active = false;     // the current step replays them
    // stage timing
    uint32_t prof_mask = 0;          // bit s: launches of stage s are bracketed by events
    int prof_every = 1;              // ... in one pool step of every prof_every (launches
    int64_t prof_tick = 0;           //     outside steps always)
    bool prof_gate = true;           // the current launches are timed
    struct Rec { hipEvent_t a, b; int stage; int64_t items; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare_events;
};

struct gtqa_state {
    gtqa_pool* pool;
    int slot;
};

namespace {

int hip_ok(hipError_t e) { return e == hipSuccess ? GTQA_OK : GTQA_ERR_HIP; }

hipEvent_t take_event(gtqa_pool* p) {
    if (!p->spare_events.empty()) {
        hipEvent_t e = p->spare_events.back();
        p->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Runs `launch` (returns 0 on success), bracketed by events when timing is on.
template <typename F>
int timed(gtqa_pool* p, int stage, int64_t items, F&& launch) {
    if (!((p->prof_mask >> stage) & 1u) || items <= 0 || !p->prof_gate) return launch() ? GTQA_ERR_HIP : GTQA_OK;
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) return GTQA_ERR_HIP;
    if (hipEventRecord(a, p->stream) != hipSuccess) return GTQA_ERR_HIP;
    const int rc = launch();
    if (hipEventRecord(b, p->stream) != hipSuccess) return GTQA_ERR_HIP;
    p->recs.push_back({a, b, stage, items});
    return rc ? GTQA_ERR_HIP : GTQA_OK;
}

void* dev_alloc(gtqa_pool* p, size_t bytes) {
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~size_t(255);
    void* ptr = nullptr;
    if (p->has_alloc) {
        ptr = p->alloc.alloc(bytes, p->alloc.ctx);
        if (!ptr) std::fprintf(stderr, "gtqa: allocator callback returned NULL for %zu bytes\n", bytes);
    } else {
        const hipError_t err = hipMalloc(&ptr, bytes);
        if (err != hipSuccess) {
            std::fprintf(stderr, "gtqa: hipMalloc(%zu) failed: %s\n", bytes, hipGetErrorString(err));
            ptr = nullptr;
        }
    }
    if (ptr) p->blocks.push_back(ptr);
    return ptr;
}

void drop_events(gtqa_pool* p) {
    for (auto& r : p->recs) {
        p->spare_events.push_back(r.a);
        p->spare_events.push_back(r.b);
    }
    p->recs.clear();
}

void drop_graphs(gtqa_pool* p) {
    for (auto& g : p->g_head) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    if (p->g_sweep) (void)hipGraphExecDestroy(p->g_sweep);
    if (p->g_tail) (void)hipGraphExecDestroy(p->g_tail);
    p->g_sweep = p->g_tail = nullptr;
    p->graphs_ok = false;
    p->graph_key.clear();
}

void release_all(gtqa_pool* p) {
    drop_graphs(p);
    drop_events(p);
    for (hipEvent_t e : p->spare_events) (void)hipEventDestroy(e);
    p->spare_events.clear();
    if (p->ev_rb) (void)hipEventDestroy(p->ev_rb);
    p->ev_rb = nullptr;
    for (void* b : p->blocks) {
        if (p->has_alloc) p->alloc.free(b, p->alloc.ctx);
        else (void)hipFree(b);
    }
    p->blocks.clear();
    if (p->h_notdone) (void)hipHostFree(p->h_notdone);
    p->h_notdone = nullptr;
    p->h_counts = nullptr;
}

int check_options(const gtqa_options* o) {
    if (!o) return GTQA_ERR_ARG;
    if (!gtqa::chi_supported(o->chi)) return GTQA_ERR_UNSUPPORTED;
    if (o->precision != GTQA_FP64 && o->precision != GTQA_MIXED) return GTQA_ERR_ARG;
    if (o->bp_max_sweeps < 1 || !std::isfinite(o->bp_tol)) return GTQA_ERR_ARG;
    if (!(o->svd_rel_cutoff >= 0.0) || !(o->eig_rel_cutoff >= 0.0)) return GTQA_ERR_ARG;
    if (o->regauge_policy < 0 || o->regauge_policy > 3) return GTQA_ERR_ARG;
    if (!std::isfinite(o->residual_max)) return GTQA_ERR_ARG;
    if (o->launch_mode != GTQA_LAUNCH_DIRECT && o->launch_mode != GTQA_LAUNCH_GRAPH) return GTQA_ERR_ARG;
    if (o->bp_schedule != GTQA_BP_COLOUR_ORDERED && o->bp_schedule != GTQA_BP_FLOODING) return GTQA_ERR_ARG;
    return GTQA_OK;
}

// Validates the graph, couplings and colouring; fills the colouring.
int validate_instance(const gtqa_instance* in, std::vector<uint8_t>& colour, int* ncol) {
    if (!in || in->n <= 0 || in->n_edges < 0) return GTQA_ERR_ARG;
    if (in->n_edges > 0 && (!in->edges || !in->J)) return GTQA_ERR_ARG;
    if (!in->h) return GTQA_ERR_ARG;
    const int n = in->n, m = in->n_edges;
    std::vector<int> deg(n, 0);
    for (int e = 0; e < m; ++e) {
        const int u = in->edges[2 * e], v = in->edges[2 * e + 1];
        if (u < 0 || v >= n || u >= v) return GTQA_ERR_GRAPH;
        if (e > 0) {
            const int pu = in->edges[2 * e - 2], pv = in->edges[2 * e - 1];
            if (pu > u || (pu == u && pv >= v)) return GTQA_ERR_GRAPH;   // sorted, no repeats
        }
        if (++deg[u] > 3 || ++deg[v] > 3) return GTQA_ERR_GRAPH;
        if (!std::isfinite(in->J[e])) return GTQA_ERR_NUMERIC;
    }
    for (int a = 0; a < n; ++a) {
        if (deg[a] == 0) return GTQA_ERR_GRAPH;
        if (!std::isfinite(in->h[a])) return GTQA_ERR_NUMERIC;
    }
    colour.assign(m, 0);
    if (in->colour) {
        int used = 0;
        std::vector<int> seen((size_t)n * kMaxColours, 0);
        for (int e = 0; e < m; ++e) {
            const int c = in->colour[e];
            if (c >= kMaxColours) return GTQA_ERR_GRAPH;
            for (int s = 0; s < 2; ++s) {
                int& f = seen[(size_t)in->edges[2 * e + s] * kMaxColours + c];
                if (f) return GTQA_ERR_GRAPH;
                f = 1;
            }
            colour[e] = (uint8_t)c;
            used = std::max(used, c + 1);
        }
        *ncol = used;
    } else {
        MisraGries mg(n, m, in->edges);
        const int used = mg.run(colour.data());
        if (used < 0) return GTQA_ERR_GRAPH;
        *ncol = used;
    }
    return GTQA_OK;
}

template <typename T>
int upload(T* dst, const T* src, size_t count, hipStream_t s) {
    if (count == 0) return GTQA_OK;
    return hip_ok(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s));
}

// Builds (or reuses) the work lists for stepping `slots`.
int prepare_plan(gtqa_pool* p, const int32_t* slots, int count) {
    std::vector<int32_t> key(slots, slots + count);
    if (key == p->plan_key) return GTQA_OK;
    // the work lists are rewritten in place: captured launches of the old
    // plan (list offsets and lengths) are stale even if the key recurs
    drop_graphs(p);
    std::vector<int32_t> lists;
    int ncol = 0;
    for (int i = 0; i < count; ++i) ncol = std::max(ncol, p->slots[slots[i]].ncol);
    for (int c = 0; c < ncol; ++c) {
        p->off_cls[c] = (int64_t)lists.size();
        for (int i = 0; i < count; ++i) {
            const SlotInfo& si = p->slots[slots[i]];
            if (c < si.ncol) lists.insert(lists.end(), si.cls[c].begin(), si.cls[c].end());
        }
    }
    p->off_cls[ncol] = (int64_t)lists.size();
    p->off_alle = (int64_t)lists.size();
    for (int i = 0; i < count; ++i) {
        const SlotInfo& si = p->slots[slots[i]];
        for (int64_t e = 0; e < si.ne; ++e) lists.push_back((int32_t)(si.e0 + e));
    }
    p->n_alle = (int64_t)lists.size() - p->off_alle;
    p->off_allv = (int64_t)lists.size();
    for (int i = 0; i < count; ++i) {
        const SlotInfo& si = p->slots[slots[i]];
        for (int64_t a = 0; a < si.nv; ++a) lists.push_back((int32_t)(si.v0 + a));
    }
    p->n_allv = (int64_t)lists.size() - p->off_allv;
    p->off_slots = (int64_t)lists.size();
    lists.insert(lists.end(), slots, slots + count);
    const int64_t cap = 3 * p->maxE + p->maxV + p->maxS + 16;
    if ((int64_t)lists.size() > cap) return GTQA_ERR_ARG;
    int rc = upload(p->lists, lists.data(), lists.size(), p->stream);
    if (rc) return rc;
    // per-slot segments of every class list (for compaction between sweeps)
    std::vector<int32_t> seg((size_t)std::max(ncol, 1) * count * 2, 0);
    for (int c = 0; c < ncol; ++c) {
        int32_t o = 0;
        for (int i = 0; i < count; ++i) {
            const SlotInfo& si = p->slots[slots[i]];
            const int32_t len = c < si.ncol ? (int32_t)si.cls[c].size() : 0;
            seg[((size_t)c * count + i) * 2] = o;
            seg[((size_t)c * count + i) * 2 + 1] = len;
            o += len;
        }
    }
    rc = upload(p->seg, seg.data(), seg.size(), p->stream);
    if (rc) return rc;
    std::vector<int64_t> coff(p->off_cls, p->off_cls + kMaxColours + 1);
    rc = upload(p->d_cls_off, coff.data(), coff.size(), p->stream);
    if (rc) return rc;
    if (gtqa::launch_bp_records(p->dp, p->lists, (int)p->off_cls[ncol], p->crec, p->stream)) return GTQA_ERR_HIP;
    rc = hip_ok(hipStreamSynchronize(p->stream));
    if (rc) return rc;
    p->plan_ncol = ncol;
    p->plan_key = key;
    return GTQA_OK;
}

// One uncompacted sweep of every class (first: warm start for the classes
// not yet visited), the zeroing of the stop-test counters and their
// reduction; with readback also the copy of the counters to the host.  This
// is the fixed part of a sweep that the graph path captures.
int sweep_launches(gtqa_pool* p, int count, bool first, bool readback) {
    const int chi = p->chi, prec = p->prec;
    const DevPool& d = p->dp;
    hipStream_t s = p->stream;
    const int32_t* slots = p->lists + p->off_slots;
    if (d.bp_flood && !first) {
        for (int c = 0; c < p->plan_ncol; ++c) {
            const int64_t o = p->off_cls[c], n = p->off_cls[c + 1] - o;
            if (gtqa::launch_bp_snapshot(chi, prec, d, p->crec + 3 * o, (int)n, s)) return GTQA_ERR_HIP;
        }
    }
    for (int c = 0; c < p->plan_ncol; ++c) {
        const int64_t o = p->off_cls[c], n = p->off_cls[c + 1] - o;
        if (gtqa::launch_bp_sweep_class(chi, prec, d, p->crec + 3 * o, (int)n, first ? 1 : 0, c, nullptr, s))
            return GTQA_ERR_HIP;
    }
    if (gtqa::launch_zero_i32(p->d_notdone, first ? 4 : 2, s)) return GTQA_ERR_HIP;
    if (gtqa::launch_bp_reduce(d, slots, count, p->d_notdone, 0, p->opt.bp_max_sweeps, s)) return GTQA_ERR_HIP;
    if (readback &&
        hipMemcpyAsync(p->h_notdone, p->d_notdone, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return GTQA_ERR_HIP;
    return GTQA_OK;
}

// BP sweeps (Alg. 1) for the slots active in the current phase; returns
// whether every slot converged before max_sweeps.
// With bp_tol > 0 the stop test runs on the device after every sweep (per
// slot: converged, still sweeping, capped at max_sweeps, or undecided when
// its distance bounds straddle the tolerance).  Before the first read-back
// the host enqueues as many sweeps as the quickest slot of the pool's
// previous re-gauging needed (before any slot stops there is nothing to
// compact, and sweeps enqueued after every slot stopped exit at once); then
// one sweep per read-back, with the class lists compacted to the slots still
// sweeping.  At each read-back the exact trace norms settle the undecided
// slots, which sweep no further until then, so every slot takes exactly the
// sweeps and stop decisions of one read-back per sweep.  With bp_tol <= 0 exactly
// max_sweeps sweeps run with no read-back; want_exact computes the exact
// distance of the last sweep for reporting.
// spec_tail (may be null): launches Alg. 2 gated on the stop-test counters;
// it is enqueued right behind the first read-back's copy, so the GPU runs it
// while the host waits for that copy alone.  *tail_done tells whether it ran
// (every slot stopped at that read-back, none undecided); otherwise its
// launches returned at once and their timing records are dropped.
// *first_done: every slot stopped at the first read-back.
int bp_loop(gtqa_pool* p, int count, int max_sweeps, bool want_exact, bool* converged_out,
            bool head_done = false, bool warm_first = true, int (*spec_tail)(gtqa_pool*, const int32_t*) = nullptr,
            bool* tail_done = nullptr, bool* first_done = nullptr, bool cleared4 = false) {
    const int chi = p->chi, prec = p->prec;
    const DevPool& d = p->dp;
    hipStream_t s = p->stream;
    const int32_t* slots = p->lists + p->off_slots;
    const int32_t* alle = p->lists + p->off_alle;
    const bool check = d.bp_tol > 0.0;
    if (tail_done) *tail_done = false;
    if (first_done) *first_done = false;
    int32_t* cnt = p->d_notdone;
    int32_t* hc = p->h_notdone + 4 + kMaxColours;     // pinned mirror of the four counters
    auto sync_read = [&](int32_t* dst, const int32_t* src, int n) {
        return hipMemcpyAsync(dst, src, n * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
               hipStreamSynchronize(s) != hipSuccess;
    };
    bool compacted = false;     // class lists replaced by the compacted ones
    // gated: a sweep enqueued ahead of the read-back, skipped on the device
    // once the previous stop test left no slot sweeping; fresh: the stop-test
    // counter is still zero from the last clear (saves a launch)
    auto launch_sweep = [&](bool first, bool force, bool gated, bool fresh = false) -> int {
        // flooding: every class's messages of the previous iterate, before any class updates
        for (int c = 0; d.bp_flood && !first && c < p->plan_ncol; ++c) {
            const int64_t o = p->off_cls[c];
            const int64_t n = compacted ? p->h_counts[c] : p->off_cls[c + 1] - o;
            const int4* rec = (compacted ? p->ccrec : p->crec) + 3 * o;
            if (gtqa::launch_bp_snapshot(chi, prec, d, rec, (int)n, s)) return GTQA_ERR_HIP;
        }
        for (int c = 0; c < p->plan_ncol; ++c) {
            const int64_t o = p->off_cls[c];
            const int64_t n = compacted ? p->h_counts[c] : p->off_cls[c + 1] - o;
            const int4* rec = (compacted ? p->ccrec : p->crec) + 3 * o;
            if (timed(p, GTQA_STAGE_BP_SWEEP, n, [&] {
                    return gtqa::launch_bp_sweep_class(chi, prec, d, rec, (int)n, first, c, gated ? cnt : nullptr, s);
                }))
                return GTQA_ERR_HIP;
        }
        if (!fresh && gtqa::launch_zero_i32(cnt, 1, s)) return GTQA_ERR_HIP;
        if (timed(p, GTQA_STAGE_BP_REDUCE, count, [&] {
                return gtqa::launch_bp_reduce(d, slots, count, cnt, force ? 1 : 0, max_sweeps, s);
            }))
            return GTQA_ERR_HIP;
        return GTQA_OK;
    };
    auto exact_pass = [&]() -> int {
        if (timed(p, GTQA_STAGE_BP_REDUCE, p->n_alle, [&] {
                return gtqa::launch_bp_exact(chi, prec, d, alle, (int)p->n_alle, 0, s);
            }) ||
            gtqa::launch_bp_reduce_exact(d, slots, count, cnt, 0, max_sweeps, s))
            return GTQA_ERR_HIP;
        return GTQA_OK;
    };

    if (!check) {
        // fixed sweep count: no stop test, no read-back
        if (!cleared4 && gtqa::launch_zero_i32(cnt, 4, s)) return GTQA_ERR_HIP;
        for (int sweep = 0; sweep < max_sweeps; ++sweep) {
            const bool force = want_exact && sweep == max_sweeps - 1;
            if (launch_sweep(sweep == 0 && warm_first, force, false, sweep == 0)) return GTQA_ERR_HIP;
            if (force && exact_pass()) return GTQA_ERR_HIP;
        }
        *converged_out = true;
        return GTQA_OK;
    }

    // cleared4: the caller's phase-flag launch already zeroed the counters
    if (!head_done && !cleared4 && gtqa::launch_zero_i32(cnt, 4, s)) return GTQA_ERR_HIP;
    bool converged = false;
    int rounds = head_done ? 1 : 0;     // sweeps enqueued so far (the head graph ran the first)
    bool head_pending = head_done;      // ... and its stop test is not read back yet
    // every read-back gives each slot still sweeping at least one sweep, so
    // max_sweeps + 1 read-backs bound the loop
    for (int rb = 0; rb <= max_sweeps; ++rb) {
        // graph path: later uncompacted sweeps replay the sweep graph, one per read-back
        const bool replay = p->graphs_active && !compacted;
        if (head_pending) {
            head_pending = false;
        } else if (replay) {
            if (rounds == 0) {
                if (sweep_launches(p, count, warm_first, false)) return GTQA_ERR_HIP;
            } else if (hipGraphLaunch(p->g_sweep, s) != hipSuccess) {
                return GTQA_ERR_HIP;
            }
            ++rounds;
        } else {
            int batch = 1;
            if (!p->graphs_active) batch = std::max(1, std::min(p->spec_rounds, max_sweeps) - rounds);
            // right after the clear of all four counters, both are still zero
            const bool cleared = rounds == 0 && !head_done;
            if (!cleared && gtqa::launch_zero_i32(cnt + 1, 1, s)) return GTQA_ERR_HIP;
            for (int j = 0; j < batch; ++j, ++rounds)
                if (launch_sweep(rounds == 0 && warm_first, false, j > 0, cleared && j == 0)) return GTQA_ERR_HIP;
        }
        if (rb == 0 && spec_tail && !head_done) {
            if (!p->ev_rb && hipEventCreateWithFlags(&p->ev_rb, hipEventDisableTiming) != hipSuccess) {
                p->ev_rb = nullptr;
                return GTQA_ERR_HIP;
            }
            if (hipMemcpyAsync(hc, cnt, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipEventRecord(p->ev_rb, s) != hipSuccess)
                return GTQA_ERR_HIP;
            const size_t r0 = p->recs.size();
            if (spec_tail(p, cnt)) return GTQA_ERR_HIP;
            const size_t r1 = p->recs.size();
            if (hipEventSynchronize(p->ev_rb) != hipSuccess) return GTQA_ERR_HIP;
            if (hc[0] == 0 && hc[1] == 0) {
                *tail_done = true;
            } else {
                for (size_t i = r0; i < r1; ++i) {
                    p->spare_events.push_back(p->recs[i].a);
                    p->spare_events.push_back(p->recs[i].b);
                }
                p->recs.erase(p->recs.begin() + (std::ptrdiff_t)r0, p->recs.begin() + (std::ptrdiff_t)r1);
            }
        } else if (sync_read(hc, cnt, 4)) {
            return GTQA_ERR_HIP;
        }
        if (rb == 0 && first_done) *first_done = hc[0] == 0 && hc[1] == 0;
        if (hc[1] > 0) {
            if (exact_pass() || sync_read(hc, cnt, 4)) return GTQA_ERR_HIP;
        }
        if (hc[0] == 0) {
            converged = true;
            break;
        }
        // drop the stopped slots' edges from the next sweeps' launches
        if (count > 1 && hc[0] < count) {
            if (gtqa::launch_bp_compact(d, slots, count, p->plan_ncol, p->seg, p->d_cls_off, p->lists,
                                        p->clists, p->crec, p->ccrec, p->d_counts, p->cscratch, s))
                return GTQA_ERR_HIP;
            if (sync_read(p->h_counts, p->d_counts, p->plan_ncol)) return GTQA_ERR_HIP;
            compacted = true;
        }
    }
    if (hc[3] > 0) p->spec_rounds = std::max(1, gtqa::kSweepBias - hc[3]);
    if (want_exact) {
        // exact distance of the last sweep for every slot (reporting only)
        if (gtqa::launch_bp_exact(chi, prec, d, alle, (int)p->n_alle, 1, s) ||
            gtqa::launch_bp_reduce_exact(d, slots, count, cnt, 1, max_sweeps, s))
            return GTQA_ERR_HIP;
    }
    *converged_out = converged && hc[2] == 0;
    return GTQA_OK;
}

template <typename F>
int capture_graph(gtqa_pool* p, hipGraphExec_t* out, F&& body) {
    hipStream_t s = p->stream;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) return GTQA_ERR_HIP;
    int rc = body();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &g);
    if (rc == GTQA_OK && (e != hipSuccess || !g)) rc = GTQA_ERR_HIP;
    if (rc == GTQA_OK && hipGraphInstantiate(out, g, nullptr, nullptr, 0) != hipSuccess) rc = GTQA_ERR_HIP;
    if (g) (void)hipGraphDestroy(g);
    return rc;
}

// Captures, for the current plan, each class's head (simple update, phase
// flags, first BP sweep, stop-test reduction), one further uncompacted
// sweep, and the gauge fix (Alg. 2 + gauge apply with U_X).  The stop-test
// read-back follows each replay as a direct copy.
int ensure_graphs(gtqa_pool* p, int count) {
    if (p->graphs_ok && p->graph_key == p->plan_key) return GTQA_OK;
    drop_graphs(p);
    const int chi = p->chi, prec = p->prec;
    const DevPool& d = p->dp;
    hipStream_t s = p->stream;
    const int32_t* slots = p->lists + p->off_slots;
    int rc = GTQA_OK;
    for (int c = 0; c < p->plan_ncol && !rc; ++c) {
        const int64_t o = p->off_cls[c], n = p->off_cls[c + 1] - o;
        rc = capture_graph(p, &p->g_head[c], [&] {
            if (gtqa::launch_simple_update(chi, prec, d, p->lists + o, (int)n, s)) return GTQA_ERR_HIP;
            if (gtqa::launch_phase_flags(d, slots, count, c, s)) return GTQA_ERR_HIP;
            return sweep_launches(p, count, true, false);
        });
    }
    if (!rc) rc = capture_graph(p, &p->g_sweep, [&] { return sweep_launches(p, count, false, false); });
    if (!rc)
        rc = capture_graph(p, &p->g_tail, [&] {
            if (gtqa::launch_canonicalise(chi, prec, d, p->lists + p->off_alle, (int)p->n_alle, s)) return GTQA_ERR_HIP;
            if (gtqa::launch_gauge_apply(chi, prec, d, p->lists + p->off_allv, (int)p->n_allv, 1, s)) return GTQA_ERR_HIP;
            return GTQA_OK;
        });
    if (rc) {
        drop_graphs(p);
        return rc;
    }
    p->graph_key = p->plan_key;
    p->graphs_ok = true;
    return GTQA_OK;
}

// Alg. 2 (canonicalisation of every edge, then the gauge maps applied to
// every vertex, with U_X where the slot's step ends); gate: see DevPool
int regauge_tail(gtqa_pool* p, const int32_t* gate) {
    DevPool d = p->dp;
    d.tail_gate = gate;
    const int chi = p->chi, prec = p->prec;
    hipStream_t s = p->stream;
    const int32_t* alle = p->lists + p->off_alle;
    const int32_t* allv = p->lists + p->off_allv;
    if (timed(p, GTQA_STAGE_CANONICALISE, p->n_alle, [&] { return gtqa::launch_canonicalise(chi, prec, d, alle, (int)p->n_alle, s); })) return GTQA_ERR_HIP;
    if (timed(p, GTQA_STAGE_GAUGE_APPLY, p->n_allv, [&] { return gtqa::launch_gauge_apply(chi, prec, d, allv, (int)p->n_allv, 1, s); })) return GTQA_ERR_HIP;
    return GTQA_OK;
}

int regauge(gtqa_pool* p, int count, int phase, bool want_exact, bool* hit_cap) {
    const int32_t* slots = p->lists + p->off_slots;
    if (gtqa::launch_phase_flags(p->dp, slots, count, phase, p->stream, p->d_notdone)) return GTQA_ERR_HIP;
    bool converged = false, tail_done = false, first_done = false;
    // Alg. 2 goes ahead of the stop test's read-back when the last re-gauging
    // stopped at its first one (not when the exact distance of the last sweep
    // is wanted: that pass reads the messages after the loop)
    const bool spec = p->tail_spec && !want_exact;
    const int rc = bp_loop(p, count, p->opt.bp_max_sweeps, want_exact, &converged, false, true,
                           spec ? regauge_tail : nullptr, &tail_done, &first_done, true);
    if (rc) return rc;
    p->tail_spec = first_done;
    if (!converged) *hit_cap = true;
    if (!tail_done && regauge_tail(p, nullptr)) return GTQA_ERR_HIP;
    return GTQA_OK;
}

int collect_stats(gtqa_pool* p, const int32_t* slots, int count, gtqa_step_stats* stats, int idx);

// Vidal residual R of every planned slot into dp.sres (and R[i] if given).
int residual(gtqa_pool* p, int count, int mode, double* R) {
    const DevPool& d = p->dp;
    hipStream_t s = p->stream;
    const int32_t* slots = p->lists + p->off_slots;
    const int32_t* allv = p->lists + p->off_allv;
    if (timed(p, GTQA_STAGE_RESIDUAL, p->n_allv, [&] {
            return gtqa::launch_residual(p->chi, p->prec, d, allv, (int)p->n_allv, slots, count, mode, s);
        }))
        return GTQA_ERR_HIP;
    if (!R) return GTQA_OK;
    std::vector<double> all(p->maxS);
    if (hipMemcpyAsync(all.data(), p->sres, sizeof(double) * p->maxS, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GTQA_ERR_HIP;
    for (int i = 0; i < count; ++i) R[i] = all[p->plan_key[i]];
    return GTQA_OK;
}

// Occasional re-gauging: after colour class `phase`, only the slots whose
// residual R exceeds residual_max are re-gauged; when none does, BP and the
// gauge fix are not launched at all.  R is first bounded without an SVD
// (Frobenius and entrywise norms of each leg's deviation); the exact trace
// norms are computed only for slots whose bounds straddle residual_max, or
// for every slot when statistics are requested (they report R itself).
int regauge_adaptive(gtqa_pool* p, int count, int phase, gtqa_step_stats* stats, bool* hit_cap) {
    const DevPool& d = p->dp;
    hipStream_t s = p->stream;
    const int32_t* slots = p->lists + p->off_slots;
    std::vector<double> R(stats ? count : 0);
    int rc = residual(p, count, stats ? gtqa::RES_EXACT : gtqa::RES_BOUNDS, stats ? R.data() : nullptr);
    if (rc) return rc;
    if (stats)
        for (int i = 0; i < count; ++i)
            if (phase < 8) stats[i].residual[phase] = R[i];
    int32_t* d_cnt = p->d_notdone + 4;
    int32_t* h_cnt = p->h_notdone + 2 + kMaxColours;
    if (hipMemsetAsync(d_cnt, 0, 2 * sizeof(int32_t), s) != hipSuccess) return GTQA_ERR_HIP;
    if (gtqa::launch_phase_flags_adaptive(d, slots, count, phase, d_cnt, s)) return GTQA_ERR_HIP;
    if (hipMemcpyAsync(h_cnt, d_cnt, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GTQA_ERR_HIP;
    if (h_cnt[1] > 0) {
        rc = residual(p, count, gtqa::RES_UNDECIDED, nullptr);
        if (rc) return rc;
        if (gtqa::launch_phase_flags_adaptive_final(d, slots, count, d_cnt, s)) return GTQA_ERR_HIP;
        if (hipMemcpyAsync(h_cnt, d_cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return GTQA_ERR_HIP;
    }
    if (h_cnt[0] == 0) return GTQA_OK;
    const int32_t* alle = p->lists + p->off_alle;
    const int32_t* allv = p->lists + p->off_allv;
    bool converged = false;
    rc = bp_loop(p, count, p->opt.bp_max_sweeps, stats != nullptr, &converged);
    if (rc) return rc;
    if (!converged) *hit_cap = true;
    const int chi = p->chi, prec = p->prec;
    if (timed(p, GTQA_STAGE_CANONICALISE, p->n_alle, [&] { return gtqa::launch_canonicalise(chi, prec, d, alle, (int)p->n_alle, s); })) return GTQA_ERR_HIP;
    if (timed(p, GTQA_STAGE_GAUGE_APPLY, p->n_allv, [&] { return gtqa::launch_gauge_apply(chi, prec, d, allv, (int)p->n_allv, 1, s); })) return GTQA_ERR_HIP;
    return collect_stats(p, p->plan_key.data(), count, stats, phase);
}

int collect_stats(gtqa_pool* p, const int32_t* slots, int count, gtqa_step_stats* stats, int idx) {
    if (!stats) return GTQA_OK;
    std::vector<int32_t> sw(p->maxS), fl(p->maxS);
    std::vector<double> dist(p->maxS);
    if (hipMemcpyAsync(sw.data(), p->ssweeps, sizeof(int32_t) * p->maxS, hipMemcpyDeviceToHost,
                       p->stream) != hipSuccess)
        return GTQA_ERR_HIP;
    if (hipMemcpyAsync(fl.data(), p->sflag, sizeof(int32_t) * p->maxS, hipMemcpyDeviceToHost,
                       p->stream) != hipSuccess)
        return GTQA_ERR_HIP;
    if (hipMemcpyAsync(dist.data(), p->sdist, sizeof(double) * p->maxS, hipMemcpyDeviceToHost,
                       p->stream) != hipSuccess)
        return GTQA_ERR_HIP;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return GTQA_ERR_HIP;
    (void)idx;
    for (int i = 0; i < count; ++i) {
        gtqa_step_stats& st = stats[i];
        if (!(fl[slots[i]] & gtqa::FLAG_ACTIVE)) continue;
        if (st.n_regauges < 8) {
            st.bp_sweeps[st.n_regauges] = sw[slots[i]];
            st.bp_dist[st.n_regauges] = dist[slots[i]];
        }
        st.n_regauges += 1;
    }
    return GTQA_OK;
}

int pool_step_body(gtqa_pool* p, const int32_t* slots, const double* tz, const double* tx, int count,
                   gtqa_step_stats* stats);

// one Trotter step of `count` slots; stage timing in every prof_every-th step
int pool_step_impl(gtqa_pool* p, const int32_t* slots, const double* tz, const double* tx, int count,
                   gtqa_step_stats* stats) {
    if (!p) return GTQA_ERR_ARG;
    p->prof_gate = p->prof_mask == 0 || p->prof_tick++ % p->prof_every == 0;
    const int rc = pool_step_body(p, slots, tz, tx, count, stats);
    p->prof_gate = true;
    return rc;
}

int pool_step_body(gtqa_pool* p, const int32_t* slots, const double* tz, const double* tx, int count,
                   gtqa_step_stats* stats) {
    if (!p || !slots || !tz || !tx || count <= 0 || count > p->maxS) return GTQA_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        if (slots[i] < 0 || slots[i] >= p->maxS || !p->slots[slots[i]].used) return GTQA_ERR_STATE;
        if (!std::isfinite(tz[i]) || !std::isfinite(tx[i])) return GTQA_ERR_NUMERIC;
        for (int j = 0; j < i; ++j)
            if (slots[j] == slots[i]) return GTQA_ERR_ARG;
    }
    int rc = prepare_plan(p, slots, count);
    if (rc) return rc;
    for (int i = 0; i < count; ++i) {
        p->h_theta[2 * slots[i]] = tz[i];
        p->h_theta[2 * slots[i] + 1] = tx[i];
    }
    rc = upload(p->theta, p->h_theta.data(), p->h_theta.size(), p->stream);
    if (rc) return rc;
    if (stats) {
        for (int i = 0; i < count; ++i) {
            std::memset(&stats[i], 0, sizeof(gtqa_step_stats));
            stats[i].n_colours = p->slots[slots[i]].ncol;
        }
    }
    const int chi = p->chi, prec = p->prec;
    hipStream_t s = p->stream;
    bool hit_cap = false;
    const int pol = p->opt.regauge_policy;
    const bool use_graphs = p->opt.launch_mode == GTQA_LAUNCH_GRAPH && s != nullptr && !stats && p->prof_mask == 0 &&
                            p->dp.bp_tol > 0.0 && pol == GTQA_REGAUGE_EVERY_COLOUR;
    if (use_graphs) {
        rc = ensure_graphs(p, count);
        if (rc) return rc;
        p->graphs_active = true;
        for (int c = 0; c < p->plan_ncol; ++c) {
            if (hipGraphLaunch(p->g_head[c], s) != hipSuccess) rc = GTQA_ERR_HIP;
            bool converged = false;
            if (!rc) rc = bp_loop(p, count, p->opt.bp_max_sweeps, false, &converged, true);
            if (!rc && !converged) hit_cap = true;
            if (!rc && hipGraphLaunch(p->g_tail, s) != hipSuccess) rc = GTQA_ERR_HIP;
            if (rc) break;
        }
        p->graphs_active = false;
        if (rc) return rc;
        if (gtqa::launch_fidelity_reduce(p->dp, p->lists + p->off_slots, count, p->chi, s)) return GTQA_ERR_HIP;
        return hit_cap ? GTQA_WARN_BP_MAXITER : GTQA_OK;
    }
    for (int c = 0; c < p->plan_ncol; ++c) {
        const int64_t o = p->off_cls[c], n = p->off_cls[c + 1] - o;
        if (timed(p, GTQA_STAGE_SIMPLE_UPDATE, n, [&] { return gtqa::launch_simple_update(chi, prec, p->dp, p->lists + o, (int)n, s); })) return GTQA_ERR_HIP;
        if (pol == GTQA_REGAUGE_EVERY_COLOUR) {
            rc = regauge(p, count, c, stats != nullptr, &hit_cap);
            if (rc) return rc;
            rc = collect_stats(p, p->plan_key.data(), count, stats, c);
            if (rc) return rc;
        } else if (pol == GTQA_REGAUGE_ADAPTIVE) {
            rc = regauge_adaptive(p, count, c, stats, &hit_cap);
            if (rc) return rc;
        }
    }
    if (pol == GTQA_REGAUGE_EVERY_STEP) {
        rc = regauge(p, count, -1, stats != nullptr, &hit_cap);
        if (rc) return rc;
        rc = collect_stats(p, p->plan_key.data(), count, stats, -1);
        if (rc) return rc;
    } else if (pol == GTQA_REGAUGE_NEVER || pol == GTQA_REGAUGE_ADAPTIVE) {
        if (timed(p, GTQA_STAGE_X_LAYER, p->n_allv, [&] { return gtqa::launch_x_layer(chi, prec, p->dp, p->lists + p->off_allv, (int)p->n_allv, s); }))
            return GTQA_ERR_HIP;
    }
    if (gtqa::launch_fidelity_reduce(p->dp, p->lists + p->off_slots, count, p->chi, s)) return GTQA_ERR_HIP;
    if (stats) {
        std::vector<double> fid((size_t)count * 3), ent(count);
        for (int i = 0; i < count; ++i) {
            if (hipMemcpyAsync(&fid[3 * i], p->sfid + 3 * (size_t)slots[i], 24, hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipMemcpyAsync(&ent[i], p->sent + slots[i], 8, hipMemcpyDeviceToHost, s) != hipSuccess)
                return GTQA_ERR_HIP;
        }
        if (hipStreamSynchronize(s) != hipSuccess) return GTQA_ERR_HIP;
        for (int i = 0; i < count; ++i) {
            stats[i].log_fidelity = fid[3 * i];
            stats[i].max_trunc_error = fid[3 * i + 1];
            stats[i].log_fidelity_total = fid[3 * i + 2];
            stats[i].entropy = ent[i];
        }
    }
    return hit_cap ? GTQA_WARN_BP_MAXITER : GTQA_OK;
}

int pool_readout_impl(gtqa_pool* p, int slot, uint32_t flags, double* z, double* rho, int8_t* x,
                      double* energy) {
    if (!p || slot < 0 || slot >= p->maxS || !p->slots[slot].used) return GTQA_ERR_STATE;
    const SlotInfo& si = p->slots[slot];
    // the slot's vertices are a contiguous range; build a small list
    std::vector<int32_t> verts(si.nv);
    for (int64_t a = 0; a < si.nv; ++a) verts[a] = (int32_t)(si.v0 + a);
    int32_t* dl = p->lists + (3 * p->maxE + p->maxV + p->maxS + 16);   // readout scratch list
    int rc = upload(dl, verts.data(), verts.size(), p->stream);
    if (rc) return rc;
    int32_t sl = slot;
    rc = upload(dl + si.nv, &sl, 1, p->stream);
    if (rc) return rc;
    if (gtqa::launch_readout(p->chi, p->prec, p->dp, dl, (int)si.nv,
                             (flags & GTQA_READ_FROM_MESSAGES) ? 1 : 0, p->stream))
        return GTQA_ERR_HIP;
    if (gtqa::launch_energy(p->dp, dl + si.nv, 1, p->stream)) return GTQA_ERR_HIP;
    hipStream_t s = p->stream;
    if (z && hipMemcpyAsync(z, p->zval + si.v0, sizeof(double) * si.nv, hipMemcpyDeviceToHost, s) != hipSuccess)
        return GTQA_ERR_HIP;
    if (rho && hipMemcpyAsync(rho, p->rho + si.v0 * 8, sizeof(double) * 8 * si.nv, hipMemcpyDeviceToHost, s) !=
                   hipSuccess)
        return GTQA_ERR_HIP;
    if (x && hipMemcpyAsync(x, p->xbits + si.v0, si.nv, hipMemcpyDeviceToHost, s) != hipSuccess)
        return GTQA_ERR_HIP;
    if (energy && hipMemcpyAsync(energy, p->senergy + slot, sizeof(double), hipMemcpyDeviceToHost, s) !=
                      hipSuccess)
        return GTQA_ERR_HIP;
    int32_t warn = 0;
    if (hipMemcpyAsync(&warn, p->swarn + slot, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return GTQA_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GTQA_ERR_HIP;
    return (warn & gtqa::WARN_JACOBI) ? GTQA_WARN_JACOBI_CAP : GTQA_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

void gtqa_default_options(gtqa_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->chi = 4;
    o->precision = GTQA_FP64;
    o->bp_tol = 1e-10;
    o->bp_max_sweeps = 50;
    o->svd_rel_cutoff = 1e-12;
    o->eig_rel_cutoff = 1e-14;
    o->regauge_policy = GTQA_REGAUGE_EVERY_COLOUR;
    o->residual_max = 1e-3;
    o->launch_mode = GTQA_LAUNCH_DIRECT;
    o->bp_schedule = GTQA_BP_COLOUR_ORDERED;
    o->stream = nullptr;
    o->allocator = nullptr;
}

const char* gtqa_strerror(int code) {
    switch (code) {
        case GTQA_OK: return "ok";
        case GTQA_WARN_BP_MAXITER: return "warning: BP reached its sweep cap";
        case GTQA_WARN_JACOBI_CAP: return "warning: a Jacobi solve reached its sweep cap";
        case GTQA_ERR_ARG: return "invalid argument";
        case GTQA_ERR_GRAPH: return "invalid graph or colouring";
        case GTQA_ERR_NOMEM: return "out of device memory";
        case GTQA_ERR_HIP: return "HIP runtime error";
        case GTQA_ERR_NUMERIC: return "non-finite input";
        case GTQA_ERR_STATE: return "invalid state for this call";
        case GTQA_BUSY: return "pool budget or capacity exhausted";
        case GTQA_ERR_UNSUPPORTED: return "bond dimension not built into this library";
        default: return "unknown status";
    }
}

const char* gtqa_version(void) { return "gtqa-mi355x 0.1 (gfx950)"; }

int gtqa_colour_edges(int32_t n, int32_t n_edges, const int32_t* edges, uint8_t* colour_out) {
    if (n <= 0 || n_edges < 0 || (n_edges > 0 && (!edges || !colour_out))) return GTQA_ERR_ARG;
    for (int e = 0; e < n_edges; ++e) {
        const int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v >= n || u >= v) return GTQA_ERR_GRAPH;
        if (e > 0) {
            const int pu = edges[2 * e - 2], pv = edges[2 * e - 1];
            if (pu > u || (pu == u && pv >= v)) return GTQA_ERR_GRAPH;
        }
    }
    MisraGries mg(n, n_edges, edges);
    const int used = mg.run(colour_out);
    return used < 0 ? GTQA_ERR_GRAPH : used;
}

size_t gtqa_footprint_bytes(int32_t n, int32_t n_edges, int32_t chi, int32_t precision) {
    if (n <= 0 || n_edges < 0 || chi <= 0) return 0;
    return (size_t)n * vertex_bytes(chi, precision) + (size_t)n_edges * edge_bytes(chi, precision) + 512;
}

int gtqa_pool_create(const gtqa_pool_options* po, gtqa_pool** out) {
    if (!po || !out) return GTQA_ERR_ARG;
    int rc = check_options(&po->base);
    if (rc) return rc;
    if (po->max_vertices <= 0 || po->max_edges < 0 || po->max_slots <= 0) return GTQA_ERR_ARG;
    if (po->max_vertices > INT32_MAX / 8 || po->max_edges > INT32_MAX / 8) return GTQA_ERR_ARG;
    gtqa_pool* p = new (std::nothrow) gtqa_pool();
    if (!p) return GTQA_ERR_NOMEM;
    p->opt = po->base;
    p->chi = po->base.chi;
    p->prec = po->base.precision;
    p->stream = (hipStream_t)po->base.stream;
    if (po->base.allocator) {
        p->alloc = *po->base.allocator;
        p->has_alloc = p->alloc.alloc && p->alloc.free;
        if (!p->has_alloc) { delete p; return GTQA_ERR_ARG; }
    }
    p->opt.allocator = nullptr;
    p->maxV = po->max_vertices;
    p->maxE = std::max<int64_t>(po->max_edges, 1);
    p->maxS = po->max_slots;
    const int chi = p->chi;
    const size_t cb = complex_bytes(p->prec);
    const size_t cap_bytes = (size_t)p->maxV * vertex_bytes(chi, p->prec) +
                             (size_t)p->maxE * edge_bytes(chi, p->prec) + (size_t)p->maxS * 512;
    p->budget = po->budget_bytes > 0 ? std::min<int64_t>(po->budget_bytes, (int64_t)cap_bytes)
                                     : (int64_t)cap_bytes;
    const int64_t V = p->maxV, E = p->maxE, S = p->maxS;
    bool ok = true;
    auto A = [&](size_t bytes) -> void* {
        void* q = dev_alloc(p, bytes);
        if (!q) ok = false;
        return q;
    };
    p->gam = A((size_t)V * 2 * chi * chi * chi * cb);
    p->lam = (double*)A((size_t)E * chi * 8);
    p->msg = A((size_t)E * 2 * chi * chi * cb);
    p->xg = A((size_t)E * 2 * chi * chi * cb);
    p->vedge = (int32_t*)A((size_t)V * 3 * 4);
    p->eend = (int32_t*)A((size_t)E * 2 * 4);
    p->eleg = (int32_t*)A((size_t)E * 2 * 4);
    p->bpmeta = (int4*)A((size_t)E * 2 * sizeof(int4));
    p->vmeta = (int4*)A((size_t)V * sizeof(int4));
    p->eslot = (int32_t*)A((size_t)E * 4);
    p->vslot = (int32_t*)A((size_t)V * 4);
    p->J = (double*)A((size_t)E * 8);
    p->hD = (double*)A((size_t)V * 8);
    p->h = (double*)A((size_t)V * 8);
    p->edist = (double*)A((size_t)E * 8);
    p->edlo = (double*)A((size_t)E * 8);
    p->edexact = (double*)A((size_t)E * 8);
    p->mold = A((size_t)E * 2 * chi * chi * cb);
    p->ecol = (uint8_t*)A((size_t)E);
    p->rho = (double*)A((size_t)V * 64);
    p->zval = (double*)A((size_t)V * 8);
    p->xbits = (int8_t*)A((size_t)V);
    p->theta = (double*)A((size_t)S * 16);
    p->sflag = (int32_t*)A((size_t)S * 4);
    p->smask = (int32_t*)A((size_t)S * 4);
    p->ssweeps = (int32_t*)A((size_t)S * 4);
    p->swarn = (int32_t*)A((size_t)S * 4);
    p->stot = (int64_t*)A((size_t)S * 16);
    p->elogf = (double*)A((size_t)E * 8);
    p->efix = (int32_t*)A((size_t)E * 4);
    p->eeps = (double*)A((size_t)E * 8);
    p->sfid = (double*)A((size_t)S * 24);
    p->vres = (double*)A((size_t)V * 8);
    p->sres = (double*)A((size_t)S * 8);
    p->vres_hi = (double*)A((size_t)V * 8);
    p->sres_hi = (double*)A((size_t)S * 8);
    p->ecut = (uint8_t*)A((size_t)E);
    p->sent = (double*)A((size_t)S * 8);
    p->sbuf = (double*)A((size_t)S * 16);
    p->sdist = (double*)A((size_t)S * 8);
    p->senergy = (double*)A((size_t)S * 8);
    p->s_e0 = (int32_t*)A((size_t)S * 4);
    p->s_ne = (int32_t*)A((size_t)S * 4);
    p->s_v0 = (int32_t*)A((size_t)S * 4);
    p->s_nv = (int32_t*)A((size_t)S * 4);
    p->lists = (int32_t*)A((size_t)(4 * E + 2 * V + 2 * S + 64) * 4);
    p->d_notdone = (int32_t*)A(256);
    p->clists = (int32_t*)A((size_t)(E + 64) * 4);
    p->crec = (int4*)A((size_t)(E + 64) * 48);
    p->ccrec = (int4*)A((size_t)(E + 64) * 48);
    p->seg = (int32_t*)A((size_t)kMaxColours * S * 2 * 4);
    p->d_cls_off = (int64_t*)A((size_t)(kMaxColours + 1) * 8);
    p->cscratch = (int32_t*)A((size_t)kMaxColours * S * 4);
    p->d_counts = (int32_t*)A((size_t)kMaxColours * 4);
    // chi >= 16: the simple update stages its QR data per chunk of edges
    p->su_chunk = gtqa::su_ws_bytes_per_edge(chi) > 0 ? (int)std::min<int64_t>(kSuChunk, E) : 0;
    p->su_ws = p->su_chunk > 0 ? (double*)A((size_t)p->su_chunk * gtqa::su_ws_bytes_per_edge(chi)) : nullptr;
    if (ok) {
        const hipError_t err = hipHostMalloc((void**)&p->h_notdone, (8 + kMaxColours) * sizeof(int32_t),
                                             hipHostMallocDefault);
        if (err != hipSuccess) {
            std::fprintf(stderr, "gtqa: hipHostMalloc failed: %s\n", hipGetErrorString(err));
            p->h_notdone = nullptr;
            ok = false;
        }
    }
    if (!ok) {
        release_all(p);
        delete p;
        return GTQA_ERR_NOMEM;
    }
    // zero the per-slot arrays
    const size_t zb[] = {(size_t)S * 4, (size_t)S * 4, (size_t)S * 4, (size_t)S * 4};
    void* zp[] = {p->sflag, p->smask, p->ssweeps, p->swarn};
    for (int i = 0; i < 4; ++i) {
        if (hipMemsetAsync(zp[i], 0, zb[i], p->stream) != hipSuccess) ok = false;
    }
    if (hipMemsetAsync(p->xg, 0, (size_t)E * 2 * chi * chi * cb, p->stream) != hipSuccess) ok = false;
    if (hipMemsetAsync(p->stot, 0, (size_t)S * 16, p->stream) != hipSuccess) ok = false;
    if (hipMemsetAsync(p->sfid, 0, (size_t)S * 24, p->stream) != hipSuccess) ok = false;
    if (hipMemsetAsync(p->elogf, 0, (size_t)E * 8, p->stream) != hipSuccess) ok = false;
    if (hipMemsetAsync(p->efix, 0, (size_t)E * 4, p->stream) != hipSuccess) ok = false;
    if (hipMemsetAsync(p->eeps, 0, (size_t)E * 8, p->stream) != hipSuccess) ok = false;
    if (!ok) {
        release_all(p);
        delete p;
        return GTQA_ERR_HIP;
    }
    p->h_counts = p->h_notdone + 2;
    p->slots.assign(S, SlotInfo());
    p->vr.reset(V);
    p->er.reset(E);
    p->h_theta.assign((size_t)S * 2, 0.0);
    DevPool& d = p->dp;
    d.gam = p->gam; d.lam = p->lam; d.msg = p->msg; d.xg = p->xg;
    d.vedge = p->vedge; d.eend = p->eend; d.eleg = p->eleg; d.bpmeta = p->bpmeta; d.vmeta = p->vmeta; d.J = p->J; d.hD = p->hD; d.h = p->h;
    d.eslot = p->eslot; d.vslot = p->vslot; d.edist = p->edist; d.rho = p->rho; d.zval = p->zval;
    d.edlo = p->edlo; d.edexact = p->edexact; d.mold = p->mold; d.ecol = p->ecol;
    d.theta = p->theta; d.sflag = p->sflag; d.smask = p->smask; d.ssweeps = p->ssweeps;
    d.sdist = p->sdist; d.s_e0 = p->s_e0; d.s_ne = p->s_ne; d.s_v0 = p->s_v0; d.s_nv = p->s_nv;
    d.swarn = p->swarn; d.senergy = p->senergy; d.xbits = p->xbits; d.stot = p->stot;
    d.elogf = p->elogf; d.eeps = p->eeps; d.sfid = p->sfid; d.efix = p->efix;
    d.vres = p->vres; d.sres = p->sres; d.vres_hi = p->vres_hi; d.sres_hi = p->sres_hi;
    d.ecut = p->ecut; d.sent = p->sent;
    d.res_max = p->opt.residual_max;
    d.svd_cut = p->opt.svd_rel_cutoff;
    d.eig_cut = p->opt.eig_rel_cutoff;
    d.bp_tol = p->opt.bp_tol;
    d.bp_flood = p->opt.bp_schedule == GTQA_BP_FLOODING ? 1 : 0;
    d.su_ws = p->su_ws;
    d.su_chunk = p->su_chunk;
    *out = p;
    return GTQA_OK;
}

int gtqa_pool_admit(gtqa_pool* p, const gtqa_instance* in, int32_t* slot_out) {
    if (!p || !in || !slot_out) return GTQA_ERR_ARG;
    std::vector<uint8_t> colour;
    int ncol = 0;
    int rc = validate_instance(in, colour, &ncol);
    if (rc) return rc;
    if (ncol > kMaxColours) return GTQA_ERR_GRAPH;
    const int n = in->n, m = in->n_edges;
    const size_t fp = gtqa_footprint_bytes(n, m, p->chi, p->prec);
    if (p->used_bytes + (int64_t)fp > p->budget) return GTQA_BUSY;
    int slot = -1;
    for (int s = 0; s < p->maxS; ++s)
        if (!p->slots[s].used) { slot = s; break; }
    if (slot < 0) return GTQA_BUSY;
    const int64_t v0 = p->vr.take(n);
    if (v0 < 0) return GTQA_BUSY;
    const int64_t e0 = p->er.take(m);
    if (e0 < 0) {
        p->vr.give(v0, n);
        return GTQA_BUSY;
    }
    // tables
    std::vector<int32_t> vedge((size_t)n * 3, -1), eend((size_t)m * 2), eleg((size_t)m * 2), eslot(m, slot),
        vslot(n, slot);
    std::vector<int> deg(n, 0);
    for (int e = 0; e < m; ++e) {   // edges sorted: each vertex's legs come in ascending id
        const int u = in->edges[2 * e], v = in->edges[2 * e + 1];
        eleg[2 * e] = deg[u];
        eleg[2 * e + 1] = deg[v];
        vedge[(size_t)u * 3 + deg[u]++] = (int32_t)(e0 + e);
        vedge[(size_t)v * 3 + deg[v]++] = (int32_t)(e0 + e);
        eend[2 * e] = (int32_t)(v0 + u);
        eend[2 * e + 1] = (int32_t)(v0 + v);
    }
    // BP metadata per direction: the vertex the message leaves, the indices of
    // the messages arriving there on its two other legs and their colours
    std::vector<int4> bpm((size_t)m * 2);
    for (int e = 0; e < m; ++e) {
        for (int d = 0; d < 2; ++d) {
            const int a = in->edges[2 * e + d];
            const int pleg = eleg[2 * e + d];
            int inc[2] = {-1, -1}, col[2] = {255, 255}, k = 0;
            for (int lg = 0; lg < 3; ++lg) {
                if (lg == pleg) continue;
                const int32_t ge = vedge[(size_t)a * 3 + lg];
                if (ge >= 0) {
                    const int le = (int)(ge - e0);
                    const int dir = (in->edges[2 * le] == a) ? 1 : 0;   // the message travelling to a
                    inc[k] = (int)(2 * ge + dir);
                    col[k] = colour[le];
                }
                ++k;
            }
            bpm[(size_t)2 * e + d] = make_int4((int)(v0 + a), inc[0], inc[1], pleg | (col[0] << 8) | (col[1] << 16));
        }
    }
    // gauge-apply metadata: per vertex the gauge map of each leg (its edge's
    // side at this vertex) and the slot
    std::vector<int4> vmm(n);
    for (int a = 0; a < n; ++a) {
        int xi[3] = {-1, -1, -1};
        for (int lg = 0; lg < 3; ++lg) {
            const int32_t ge = vedge[(size_t)a * 3 + lg];
            if (ge < 0) continue;
            const int le = (int)(ge - e0);
            xi[lg] = (int)(2 * ge + (in->edges[2 * le] == a ? 0 : 1));
        }
        vmm[a] = make_int4(xi[0], xi[1], xi[2], slot);
    }
    std::vector<double> hD(n), hh(in->h, in->h + n), Jv(in->J, in->J + m);
    for (int a = 0; a < n; ++a) hD[a] = in->h[a] / deg[a];
    SlotInfo& si = p->slots[slot];
    si = SlotInfo();
    si.used = true;
    si.v0 = v0; si.nv = n; si.e0 = e0; si.ne = m;
    si.ncol = ncol;
    si.bytes = fp;
    si.cls.assign(ncol, {});
    for (int e = 0; e < m; ++e) si.cls[colour[e]].push_back((int32_t)(e0 + e));
    si.edges.assign(in->edges, in->edges + 2 * (size_t)m);
    si.mask = 0;
    for (int c = 0; c < ncol; ++c)
        if (!si.cls[c].empty()) si.mask |= (1 << c);
    hipStream_t s = p->stream;
    int32_t meta[5] = {(int32_t)e0, (int32_t)m, (int32_t)v0, (int32_t)n, si.mask};
    rc = GTQA_OK;
    rc = rc ? rc : upload(p->vedge + v0 * 3, vedge.data(), vedge.size(), s);
    rc = rc ? rc : upload(p->eend + e0 * 2, eend.data(), eend.size(), s);
    rc = rc ? rc : upload(p->eleg + e0 * 2, eleg.data(), eleg.size(), s);
    rc = rc ? rc : upload(p->bpmeta + e0 * 2, bpm.data(), bpm.size(), s);
    rc = rc ? rc : upload(p->vmeta + v0, vmm.data(), vmm.size(), s);
    rc = rc ? rc : upload(p->eslot + e0, eslot.data(), eslot.size(), s);
    rc = rc ? rc : upload(p->vslot + v0, vslot.data(), vslot.size(), s);
    rc = rc ? rc : upload(p->J + e0, Jv.data(), Jv.size(), s);
    rc = rc ? rc : upload(p->ecol + e0, colour.data(), colour.size(), s);
    rc = rc ? rc : upload(p->hD + v0, hD.data(), hD.size(), s);
    rc = rc ? rc : upload(p->h + v0, hh.data(), hh.size(), s);
    rc = rc ? rc : upload(p->s_e0 + slot, &meta[0], 1, s);
    rc = rc ? rc : upload(p->s_ne + slot, &meta[1], 1, s);
    rc = rc ? rc : upload(p->s_v0 + slot, &meta[2], 1, s);
    rc = rc ? rc : upload(p->s_nv + slot, &meta[3], 1, s);
    rc = rc ? rc : upload(p->smask + slot, &meta[4], 1, s);
    if (!rc && hipMemsetAsync(p->swarn + slot, 0, 4, s) != hipSuccess) rc = GTQA_ERR_HIP;
    if (!rc && hipMemsetAsync(p->stot + 2 * slot, 0, 16, s) != hipSuccess) rc = GTQA_ERR_HIP;
    if (!rc && hipMemsetAsync(p->sfid + 3 * slot, 0, 24, s) != hipSuccess) rc = GTQA_ERR_HIP;
    if (!rc && hipMemsetAsync(p->sent + slot, 0, 8, s) != hipSuccess) rc = GTQA_ERR_HIP;
    if (!rc && m > 0 && hipMemsetAsync(p->ecut + e0, 0, (size_t)m, s) != hipSuccess) rc = GTQA_ERR_HIP;
    // initial state |+>^N, every bond of dimension 1
    std::vector<int32_t> vl(n), el(m);
    for (int a = 0; a < n; ++a) vl[a] = (int32_t)(v0 + a);
    for (int e = 0; e < m; ++e) el[e] = (int32_t)(e0 + e);
    int32_t* scratch = p->lists + (3 * p->maxE + p->maxV + p->maxS + 16);
    rc = rc ? rc : upload(scratch, vl.data(), vl.size(), s);
    rc = rc ? rc : upload(scratch + n, el.data(), el.size(), s);
    if (!rc && gtqa::launch_init_plus(p->chi, p->prec, p->dp, scratch, n, scratch + n, m, s)) rc = GTQA_ERR_HIP;
    if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = GTQA_ERR_HIP;
    if (rc) {
        p->vr.give(v0, n);
        p->er.give(e0, m);
        si = SlotInfo();
        return rc;
    }
    p->used_bytes += (int64_t)fp;
    p->resident += 1;
    p->plan_key.clear();
    *slot_out = slot;
    return GTQA_OK;
}

int gtqa_pool_step(gtqa_pool* p, const int32_t* slots, const double* tz, const double* tx, int32_t count,
                   gtqa_step_stats* stats) {
    return pool_step_impl(p, slots, tz, tx, count, stats);
}

int gtqa_pool_readout(gtqa_pool* p, int32_t slot, double* z, double* rho, int8_t* x, double* energy) {
    return pool_readout_impl(p, slot, GTQA_READ_FROM_VIDAL, z, rho, x, energy);
}

int gtqa_pool_release(gtqa_pool* p, int32_t slot) {
    if (!p || slot < 0 || slot >= p->maxS || !p->slots[slot].used) return GTQA_ERR_STATE;
    // work already enqueued for this slot must finish before its ranges are reused
    if (hipStreamSynchronize(p->stream) != hipSuccess) return GTQA_ERR_HIP;
    SlotInfo& si = p->slots[slot];
    p->vr.give(si.v0, si.nv);
    p->er.give(si.e0, si.ne);
    p->used_bytes -= (int64_t)si.bytes;
    p->resident -= 1;
    si = SlotInfo();
    p->plan_key.clear();
    return GTQA_OK;
}

int64_t gtqa_pool_free_bytes(const gtqa_pool* p) { return p ? p->budget - p->used_bytes : 0; }
int32_t gtqa_pool_resident(const gtqa_pool* p) { return p ? p->resident : 0; }

void gtqa_pool_free(gtqa_pool* p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->stream);
    release_all(p);
    delete p;
}

int gtqa_init_state(const gtqa_instance* in, const gtqa_options* opt, gtqa_state** out) {
    if (!in || !opt || !out) return GTQA_ERR_ARG;
    int rc = check_options(opt);
    if (rc) return rc;
    {
        // validate before touching the device
        std::vector<uint8_t> colour;
        int ncol = 0;
        rc = validate_instance(in, colour, &ncol);
        if (rc) return rc;
    }
    gtqa_pool_options po;
    std::memset(&po, 0, sizeof(po));
    po.base = *opt;
    po.max_vertices = std::max(in->n, 1);
    po.max_edges = std::max(in->n_edges, 1);
    po.max_slots = 1;
    po.budget_bytes = 0;
    gtqa_pool* p = nullptr;
    rc = gtqa_pool_create(&po, &p);
    if (rc) return rc;
    int32_t slot = -1;
    rc = gtqa_pool_admit(p, in, &slot);
    if (rc) {
        gtqa_pool_free(p);
        return rc == GTQA_BUSY ? GTQA_ERR_NOMEM : rc;
    }
    gtqa_state* st = new (std::nothrow) gtqa_state{p, slot};
    if (!st) {
        gtqa_pool_free(p);
        return GTQA_ERR_NOMEM;
    }
    *out = st;
    return GTQA_OK;
}

int gtqa_trotter_step(gtqa_state* st, double theta_z, double theta_x, gtqa_step_stats* stats) {
    if (!st) return GTQA_ERR_ARG;
    const int32_t slot = st->slot;
    return pool_step_impl(st->pool, &slot, &theta_z, &theta_x, 1, stats);
}

int gtqa_bp_converge(gtqa_state* st, double tol, int32_t max_sweeps, uint32_t flags, uint64_t seed,
                     int32_t* sweeps_out, double* dist_out) {
    if (!st || max_sweeps < 1 || !std::isfinite(tol)) return GTQA_ERR_ARG;
    if (flags & ~(GTQA_BP_REGAUGE | GTQA_BP_RANDOM)) return GTQA_ERR_ARG;
    gtqa_pool* p = st->pool;
    const int32_t slot = st->slot;
    int rc = prepare_plan(p, &slot, 1);
    if (rc) return rc;
    const gtqa_options saved = p->opt;
    p->opt.bp_tol = tol;
    p->opt.bp_max_sweeps = max_sweeps;
    p->dp.bp_tol = tol;
    const int chi = p->chi, prec = p->prec;
    const DevPool& d = p->dp;
    hipStream_t s = p->stream;
    const int32_t* slots = p->lists + p->off_slots;
    bool cap = false;
    rc = gtqa::launch_phase_flags(d, slots, 1, -1, s) ? GTQA_ERR_HIP : GTQA_OK;
    const bool random = (flags & GTQA_BP_RANDOM) != 0;
    if (!rc && random &&
        gtqa::launch_random_messages(chi, prec, d, p->lists + p->off_alle, (int)p->n_alle, seed, s))
        rc = GTQA_ERR_HIP;
    bool converged = false;
    if (!rc) rc = bp_loop(p, 1, max_sweeps, true, &converged, false, !random);
    if (!rc && tol > 0.0 && !converged) cap = true;
    if (!rc && (sweeps_out || dist_out)) {
        int32_t sw = 0;
        double dist = 0.0;
        if (hipMemcpyAsync(&sw, p->ssweeps + slot, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&dist, p->sdist + slot, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = GTQA_ERR_HIP;
        if (sweeps_out) *sweeps_out = sw;
        if (dist_out) *dist_out = dist;
    }
    if (!rc && (flags & GTQA_BP_REGAUGE)) {
        // Alg. 2 on the converged messages, without the mixing layer: the
        // phase-0 flags mark the slot active (class 0 is never empty) and the
        // gauge kernel is told not to fuse U_X.
        if (gtqa::launch_phase_flags(d, slots, 1, 0, s)) rc = GTQA_ERR_HIP;
        if (!rc && gtqa::launch_canonicalise(chi, prec, d, p->lists + p->off_alle, (int)p->n_alle, s))
            rc = GTQA_ERR_HIP;
        if (!rc && gtqa::launch_gauge_apply(chi, prec, d, p->lists + p->off_allv, (int)p->n_allv, 0, s))
            rc = GTQA_ERR_HIP;
    }
    p->opt = saved;
    p->dp.bp_tol = saved.bp_tol;
    if (rc) return rc;
    return cap ? GTQA_WARN_BP_MAXITER : GTQA_OK;
}

int gtqa_set_tuning(int32_t knob, int32_t value) {
    gtqa::Tuning& t = gtqa::tuning();
    if (knob == GTQA_TUNE_SU_EDGES_PER_WAVE_CHI4) {
        if (value != 2 && value != 4) return GTQA_ERR_ARG;
        t.su_epw_chi4 = value;
        return GTQA_OK;
    }
    if (knob == GTQA_TUNE_XCD_CONTIGUOUS) {
        if (value != 0 && value != 1) return GTQA_ERR_ARG;
        t.xcd_remap = value;
        return GTQA_OK;
    }
    if (knob == GTQA_TUNE_CANON_LANES_CHI4) {
        if (value != 4 && value != 8) return GTQA_ERR_ARG;
        t.canon_lanes_chi4 = value;
        return GTQA_OK;
    }
    return GTQA_ERR_ARG;
}

int gtqa_get_tuning(int32_t knob, int32_t* value) {
    if (!value) return GTQA_ERR_ARG;
    const gtqa::Tuning& t = gtqa::tuning();
    if (knob == GTQA_TUNE_SU_EDGES_PER_WAVE_CHI4) *value = t.su_epw_chi4;
    else if (knob == GTQA_TUNE_XCD_CONTIGUOUS) *value = t.xcd_remap;
    else if (knob == GTQA_TUNE_CANON_LANES_CHI4) *value = t.canon_lanes_chi4;
    else return GTQA_ERR_ARG;
    return GTQA_OK;
}

int gtqa_pool_set_bipartition(gtqa_pool* p, int32_t slot, const uint8_t* side) {
    if (!p || !side) return GTQA_ERR_ARG;
    if (slot < 0 || slot >= p->maxS || !p->slots[slot].used) return GTQA_ERR_STATE;
    const SlotInfo& si = p->slots[slot];
    std::vector<uint8_t> cut((size_t)si.ne);
    for (int64_t e = 0; e < si.ne; ++e)
        cut[e] = (side[si.edges[2 * e]] != 0) != (side[si.edges[2 * e + 1]] != 0) ? 1 : 0;
    int rc = upload(p->ecut + si.e0, cut.data(), cut.size(), p->stream);
    if (rc) return rc;
    // buffers passed to an async copy must outlive it
    return hip_ok(hipStreamSynchronize(p->stream));
}

int gtqa_pool_entropy(gtqa_pool* p, int32_t slot, double* S) {
    if (!p || !S) return GTQA_ERR_ARG;
    if (slot < 0 || slot >= p->maxS || !p->slots[slot].used) return GTQA_ERR_STATE;
    int32_t* dl = p->lists + (3 * p->maxE + p->maxV + p->maxS + 16);   // scratch list
    int rc = upload(dl, &slot, 1, p->stream);
    if (rc) return rc;
    if (gtqa::launch_entropy(p->dp, dl, 1, p->chi, p->stream)) return GTQA_ERR_HIP;
    if (hipMemcpyAsync(S, p->sent + slot, 8, hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
        return GTQA_ERR_HIP;
    return GTQA_OK;
}

int gtqa_pool_sample(gtqa_pool* p, const int32_t* slots, int32_t count, const double* u, double tol,
                     int32_t max_sweeps, int8_t* x, double* energy, double* prob, int32_t* sweeps) {
    if (!p || !slots || !u || count <= 0 || count > p->maxS || max_sweeps < 1 || !std::isfinite(tol))
        return GTQA_ERR_ARG;
    std::vector<int64_t> off(count + 1, 0);
    for (int i = 0; i < count; ++i) {
        if (slots[i] < 0 || slots[i] >= p->maxS || !p->slots[slots[i]].used) return GTQA_ERR_STATE;
        for (int j = 0; j < i; ++j)
            if (slots[j] == slots[i]) return GTQA_ERR_ARG;
        off[i + 1] = off[i] + p->slots[slots[i]].nv;
    }
    for (int64_t k = 0; k < off[count]; ++k)
        if (!(u[k] >= 0.0 && u[k] < 1.0)) return GTQA_ERR_ARG;
    int rc = prepare_plan(p, slots, count);
    if (rc) return rc;
    const gtqa_options saved = p->opt;
    p->opt.bp_tol = tol;
    p->opt.bp_max_sweeps = max_sweeps;
    p->dp.bp_tol = tol;
    const int chi = p->chi, prec = p->prec;
    const DevPool& d = p->dp;
    hipStream_t s = p->stream;
    const int32_t* dslots = p->lists + p->off_slots;
    int32_t* dl = p->lists + (3 * p->maxE + p->maxV + p->maxS + 16);   // scratch vertex list
    double* du = p->sbuf;
    double* dprob = p->sbuf + p->maxS;
    int64_t nmax = 0;
    for (int i = 0; i < count; ++i) nmax = std::max<int64_t>(nmax, p->slots[slots[i]].nv);
    std::vector<int32_t> verts;
    std::vector<double> uh(count), ph(count);
    std::vector<int32_t> sw(p->maxS);
    bool warn = false;
    // re-gauging, then the message-form marginals of qubit q (before Alg. 2
    // moves the tensors out of the messages' gauge), then Alg. 2
    auto regauge_and_read = [&](int64_t q) -> int {
        bool conv = false;
        int r = bp_loop(p, count, max_sweeps, false, &conv);
        if (r) return r;
        if (!conv) warn = true;
        verts.clear();
        for (int i = 0; i < count; ++i) {
            const SlotInfo& si = p->slots[slots[i]];
            if (q < si.nv) verts.push_back((int32_t)(si.v0 + q));
        }
        if (!verts.empty()) {
            r = upload(dl, verts.data(), verts.size(), s);
            if (r) return r;
            if (gtqa::launch_readout(chi, prec, d, dl, (int)verts.size(), 1, s)) return GTQA_ERR_HIP;
        }
        if (gtqa::launch_canonicalise(chi, prec, d, p->lists + p->off_alle, (int)p->n_alle, s) ||
            gtqa::launch_gauge_apply(chi, prec, d, p->lists + p->off_allv, (int)p->n_allv, 0, s))
            return GTQA_ERR_HIP;
        return hip_ok(hipStreamSynchronize(s));
    };
    if (gtqa::launch_sample_flags(d, dslots, count, 0, s)) rc = GTQA_ERR_HIP;
    if (!rc) rc = regauge_and_read(0);
    for (int64_t a = 0; a < nmax && !rc; ++a) {
        for (int i = 0; i < count; ++i)
            uh[i] = a < p->slots[slots[i]].nv ? u[off[i] + a] : 0.0;
        rc = upload(du, uh.data(), uh.size(), s);
        if (!rc && gtqa::launch_sample_project(chi, prec, d, dslots, count, (int)a, du, dprob, s)) rc = GTQA_ERR_HIP;
        if (!rc && gtqa::launch_sample_flags(d, dslots, count, (int)a, s)) rc = GTQA_ERR_HIP;
        if (!rc && prob &&
            hipMemcpyAsync(ph.data(), dprob, sizeof(double) * count, hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = GTQA_ERR_HIP;
        if (!rc) rc = regauge_and_read(a + 1);
        if (!rc && sweeps &&
            (hipMemcpyAsync(sw.data(), p->ssweeps, sizeof(int32_t) * p->maxS, hipMemcpyDeviceToHost, s) !=
                 hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess))
            rc = GTQA_ERR_HIP;
        for (int i = 0; i < count && !rc; ++i) {
            if (a >= p->slots[slots[i]].nv) continue;
            if (prob) prob[off[i] + a] = ph[i];
            if (sweeps) sweeps[off[i] + a] = sw[slots[i]];
        }
    }
    if (!rc && gtqa::launch_energy(d, dslots, count, s)) rc = GTQA_ERR_HIP;
    for (int i = 0; i < count && !rc; ++i) {
        const SlotInfo& si = p->slots[slots[i]];
        if (x && hipMemcpyAsync(x + off[i], p->xbits + si.v0, si.nv, hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = GTQA_ERR_HIP;
        if (!rc && energy &&
            hipMemcpyAsync(energy + i, p->senergy + slots[i], sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
            rc = GTQA_ERR_HIP;
    }
    if (!rc) rc = hip_ok(hipStreamSynchronize(s));
    p->opt = saved;
    p->dp.bp_tol = saved.bp_tol;
    if (rc) return rc;
    return warn ? GTQA_WARN_BP_MAXITER : GTQA_OK;
}

int gtqa_sample(gtqa_state* st, const double* u, double tol, int32_t max_sweeps, int8_t* x, double* energy,
                double* prob, int32_t* sweeps) {
    if (!st) return GTQA_ERR_ARG;
    return gtqa_pool_sample(st->pool, &st->slot, 1, u, tol, max_sweeps, x, energy, prob, sweeps);
}

int gtqa_set_bipartition(gtqa_state* st, const uint8_t* side) {
    if (!st) return GTQA_ERR_ARG;
    return gtqa_pool_set_bipartition(st->pool, st->slot, side);
}

int gtqa_entropy(gtqa_state* st, double* S) {
    if (!st) return GTQA_ERR_ARG;
    return gtqa_pool_entropy(st->pool, st->slot, S);
}

int gtqa_vidal_residual(gtqa_state* st, double* R) {
    if (!st || !R) return GTQA_ERR_ARG;
    return gtqa_pool_residual(st->pool, &st->slot, 1, R);
}

int gtqa_pool_x_layer(gtqa_pool* p, const int32_t* slots, int32_t count, const double* theta_x) {
    if (!p || !slots || !theta_x || count <= 0 || count > p->maxS) return GTQA_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        if (slots[i] < 0 || slots[i] >= p->maxS || !p->slots[slots[i]].used) return GTQA_ERR_STATE;
        if (!std::isfinite(theta_x[i])) return GTQA_ERR_NUMERIC;
        for (int j = 0; j < i; ++j)
            if (slots[j] == slots[i]) return GTQA_ERR_ARG;
    }
    int rc = prepare_plan(p, slots, count);
    if (rc) return rc;
    for (int i = 0; i < count; ++i) p->h_theta[2 * slots[i] + 1] = theta_x[i];
    rc = upload(p->theta, p->h_theta.data(), p->h_theta.size(), p->stream);
    if (rc) return rc;
    const int chi = p->chi, prec = p->prec;
    hipStream_t s = p->stream;
    if (timed(p, GTQA_STAGE_X_LAYER, p->n_allv, [&] {
            return gtqa::launch_x_layer(chi, prec, p->dp, p->lists + p->off_allv, (int)p->n_allv, s);
        }))
        return GTQA_ERR_HIP;
    return GTQA_OK;
}

int gtqa_x_layer(gtqa_state* st, double theta_x) {
    if (!st) return GTQA_ERR_ARG;
    const int32_t slot = st->slot;
    return gtqa_pool_x_layer(st->pool, &slot, 1, &theta_x);
}

int gtqa_pool_residual(gtqa_pool* p, const int32_t* slots, int32_t count, double* R) {
    if (!p || !slots || !R || count <= 0 || count > p->maxS) return GTQA_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        if (slots[i] < 0 || slots[i] >= p->maxS || !p->slots[slots[i]].used) return GTQA_ERR_STATE;
        for (int j = 0; j < i; ++j)
            if (slots[j] == slots[i]) return GTQA_ERR_ARG;
    }
    const int rc = prepare_plan(p, slots, count);
    if (rc) return rc;
    return residual(p, count, gtqa::RES_EXACT, R);
}

int gtqa_readout(gtqa_state* st, uint32_t flags, double* z, double* rho, int8_t* x, double* energy) {
    if (!st) return GTQA_ERR_ARG;
    return pool_readout_impl(st->pool, st->slot, flags, z, rho, x, energy);
}

void gtqa_free_state(gtqa_state* st) {
    if (!st) return;
    gtqa_pool_free(st->pool);
    delete st;
}

int gtqa_pool_bp_totals(gtqa_pool* p, int32_t slot, int64_t* sweeps, int64_t* regauges) {
    if (!p || slot < 0 || slot >= p->maxS || !p->slots[slot].used) return GTQA_ERR_STATE;
    int64_t v[2] = {0, 0};
    if (hipMemcpyAsync(v, p->stot + 2 * slot, 16, hipMemcpyDeviceToHost, p->stream) != hipSuccess ||
        hipStreamSynchronize(p->stream) != hipSuccess)
        return GTQA_ERR_HIP;
    if (sweeps) *sweeps = v[0];
    if (regauges) *regauges = v[1];
    return GTQA_OK;
}

int gtqa_pool_profile_stages(gtqa_pool* p, uint32_t stage_mask) {
    if (!p || (stage_mask >> GTQA_N_STAGES) != 0) return GTQA_ERR_ARG;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return GTQA_ERR_HIP;
    drop_events(p);
    p->prof_mask = stage_mask;
    p->prof_tick = 0;
    return GTQA_OK;
}

int gtqa_pool_profile_sample(gtqa_pool* p, int32_t every) {
    if (!p || every < 1) return GTQA_ERR_ARG;
    p->prof_every = every;
    p->prof_tick = 0;
    return GTQA_OK;
}

int gtqa_pool_profile(gtqa_pool* p, int32_t enable) {
    return gtqa_pool_profile_stages(p, enable != 0 ? (1u << GTQA_N_STAGES) - 1u : 0u);
}

int gtqa_pool_profile_read(gtqa_pool* p, int32_t stage, int64_t* launches, double* total_ms,
                           int64_t* items) {
    if (!p || stage < 0 || stage >= GTQA_N_STAGES) return GTQA_ERR_ARG;
    if (hipStreamSynchronize(p->stream) != hipSuccess) return GTQA_ERR_HIP;
    int64_t n = 0, it = 0;
    double tot = 0.0;
    for (const auto& r : p->recs) {
        if (r.stage != stage) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return GTQA_ERR_HIP;
        tot += ms;
        n += 1;
        it += r.items;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = tot;
    if (items) *items = it;
    return GTQA_OK;
}

int gtqa_pool_set_network(gtqa_pool* p, int32_t slot, const double* gamma, const double* lam) {
    if (!p || slot < 0 || slot >= p->maxS || !p->slots[slot].used) return GTQA_ERR_STATE;
    if (!gamma || !lam) return GTQA_ERR_ARG;
    const SlotInfo& si = p->slots[slot];
    const int chi = p->chi;
    const size_t G = (size_t)2 * chi * chi * chi;
    const size_t ng = (size_t)si.nv * G * 2, nl = (size_t)si.ne * chi;
    for (size_t i = 0; i < ng; ++i)
        if (!std::isfinite(gamma[i])) return GTQA_ERR_NUMERIC;
    for (int64_t e = 0; e < si.ne; ++e) {
        for (int j = 0; j < chi; ++j) {
            const double v = lam[e * chi + j];
            if (!std::isfinite(v)) return GTQA_ERR_NUMERIC;
            if (v < 0.0 || (j > 0 && v > lam[e * chi + j - 1])) return GTQA_ERR_ARG;
        }
        if (!(lam[e * chi] > 0.0)) return GTQA_ERR_ARG;
    }
    hipStream_t s = p->stream;
    const size_t cb = complex_bytes(p->prec);
    char* dst = static_cast<char*>(p->gam) + (size_t)si.v0 * G * cb;
    std::vector<float> tmp;
    if (p->prec == GTQA_MIXED) {
        tmp.resize(ng);
        for (size_t i = 0; i < ng; ++i) tmp[i] = (float)gamma[i];
        if (hipMemcpyAsync(dst, tmp.data(), ng * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess)
            return GTQA_ERR_HIP;
    } else if (hipMemcpyAsync(dst, gamma, ng * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) {
        return GTQA_ERR_HIP;
    }
    if (hipMemcpyAsync(p->lam + si.e0 * chi, lam, nl * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return GTQA_ERR_HIP;
    return hip_ok(hipStreamSynchronize(s));
}

int gtqa_pool_get_network(gtqa_pool* p, int32_t slot, double* gamma, double* lam) {
    if (!p || slot < 0 || slot >= p->maxS || !p->slots[slot].used) return GTQA_ERR_STATE;
    const SlotInfo& si = p->slots[slot];
    const int chi = p->chi;
    const size_t G = (size_t)2 * chi * chi * chi;
    const size_t ng = (size_t)si.nv * G * 2, nl = (size_t)si.ne * chi;
    hipStream_t s = p->stream;
    const size_t cb = complex_bytes(p->prec);
    const char* src = static_cast<const char*>(p->gam) + (size_t)si.v0 * G * cb;
    std::vector<float> tmp;
    if (gamma) {
        if (p->prec == GTQA_MIXED) {
            tmp.resize(ng);
            if (hipMemcpyAsync(tmp.data(), src, ng * sizeof(float), hipMemcpyDeviceToHost, s) != hipSuccess)
                return GTQA_ERR_HIP;
        } else if (hipMemcpyAsync(gamma, src, ng * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) {
            return GTQA_ERR_HIP;
        }
    }
    if (lam && hipMemcpyAsync(lam, p->lam + si.e0 * chi, nl * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
        return GTQA_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return GTQA_ERR_HIP;
    if (gamma && p->prec == GTQA_MIXED)
        for (size_t i = 0; i < ng; ++i) gamma[i] = (double)tmp[i];
    return GTQA_OK;
}

int gtqa_set_network(gtqa_state* st, const double* gamma, const double* lam) {
    if (!st) return GTQA_ERR_ARG;
    return gtqa_pool_set_network(st->pool, st->slot, gamma, lam);
}

int gtqa_get_network(gtqa_state* st, double* gamma, double* lam) {
    if (!st) return GTQA_ERR_ARG;
    return gtqa_pool_get_network(st->pool, st->slot, gamma, lam);
}

int gtqa_bond_svd(int32_t chi, int32_t count, const double* core, double svd_rel_cutoff, double* sigma,
                  int32_t* sweeps) {
    if (!gtqa::chi_supported(chi)) return GTQA_ERR_UNSUPPORTED;
    if (count < 0 || (count > 0 && (!core || !sigma || !sweeps)) || !(svd_rel_cutoff >= 0.0) ||
        !std::isfinite(svd_rel_cutoff))
        return GTQA_ERR_ARG;
    if (count == 0) return GTQA_OK;
    const size_t N = (size_t)2 * chi;
    const size_t nc = (size_t)count * N * N * 2;
    for (size_t i = 0; i < nc; ++i)
        if (!std::isfinite(core[i])) return GTQA_ERR_NUMERIC;
    double *dcore = nullptr, *dsig = nullptr;
    int32_t* dsw = nullptr;
    int rc = GTQA_OK;
    if (hipMalloc(&dcore, nc * sizeof(double)) != hipSuccess ||
        hipMalloc(&dsig, (size_t)count * N * sizeof(double)) != hipSuccess ||
        hipMalloc(&dsw, (size_t)count * sizeof(int32_t)) != hipSuccess)
        rc = GTQA_ERR_NOMEM;
    if (!rc && hipMemcpy(dcore, core, nc * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) rc = GTQA_ERR_HIP;
    if (!rc && gtqa::launch_core_svd(chi, dcore, count, svd_rel_cutoff, dsig, dsw, nullptr)) rc = GTQA_ERR_HIP;
    if (!rc && (hipMemcpy(sigma, dsig, (size_t)count * N * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(sweeps, dsw, (size_t)count * sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess))
        rc = GTQA_ERR_HIP;
    if (dcore) (void)hipFree(dcore);
    if (dsig) (void)hipFree(dsig);
    if (dsw) (void)hipFree(dsw);
    return rc;
}

int gtqa_pool_set_bp(gtqa_pool* p, double tol, int32_t max_sweeps) {
    if (!p) return GTQA_ERR_ARG;
    if (max_sweeps < 1 || !std::isfinite(tol)) return GTQA_ERR_ARG;
    if ((tol > 0.0) != (p->dp.bp_tol > 0.0)) drop_graphs(p);   // captured sequences depend on the stop test
    p->opt.bp_tol = tol;
    p->opt.bp_max_sweeps = max_sweeps;
    p->dp.bp_tol = tol;
    return GTQA_OK;
}

}  // extern "C"
