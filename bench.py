#!/usr/bin/env python
"""Trotter gate-updates/s of the GTQA Trotter step at n=1000, chi=4 on one MI355X.

Workload: B independent random 3-regular instances (n=1000, 1500 edges,
J, h uniform on the 2^-24 grid of [-1, 1), seeds 2000+i) resident in one
pool; one bench step = one first-order Trotter step of the T=100, dt=0.05
linear-schedule anneal for all B instances (simple update of every colour
class, BP re-gauging after each class, X layer), i.e. B*1500 gate updates.
The K timed steps sit in the middle of the 2000-step anneal (the whole
anneal after W steps when K fills it): an untimed pre-roll brings every
instance to the window, its last W steps being the warm-up.

Beside the headline: comparison legs on a mid-anneal window (plain = one
instance in FP64 at BP tolerance 1e-10; batch sizes 1..256 in both
precisions; each precision also at the other's tolerance), adaptive
re-gauging, a serving run, and the oracle's CPU rate.  One JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(msg: str) -> None:
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_item(stage: str, chi: int, precision: str) -> float:
    """Minimum HBM bytes one work item of a stage must move (read + write).

    w = bytes per complex in storage, G = 2 chi^3 w (one site tensor),
    M = chi^2 w (one message), L = 8 chi (one lambda vector, FP64)."""
    w = 8 if precision == "mixed" else 16
    G = 2 * chi ** 3 * w
    M = chi * chi * w
    L = 8 * chi
    if stage == "bp_sweep":        # per edge: 2 tensors, 4 incoming + 2 old messages, 6 lambdas; write 2 messages
        return 2 * G + 6 * M + 6 * L + 2 * M + 8
    if stage == "simple_update":   # per edge: 2 tensors + 5 lambdas in, 2 tensors + 1 lambda out
        return 2 * G + 5 * L + 2 * G + L
    if stage == "canonicalise":    # per edge: 2 messages + lambda in; 2 gauge maps (storage precision) + lambda out
        return 2 * M + L + 2 * M + L
    if stage == "gauge_apply":     # per vertex: tensor + 3 gauge maps in, tensor out
        return G + 3 * M + G
    if stage == "bp_init":         # per edge: lambda in, 2 messages out
        return L + 2 * M
    return 0.0


def algorithmic_flops_per_item(stage: str, chi: int) -> float:
    """Real floating-point operations one work item needs (a complex
    multiply-add counts 8).  The Jacobi SVD is charged 6 sweeps."""
    c = chi
    if stage == "simple_update":
        qr = 4 * 8 * (c ** 4 - c ** 3 / 3.0)          # Householder QR of four chi^2 x chi blocks
        core = 8 * (2 * c) ** 2 * c                     # 2chi x 2chi core from the R factors
        n = 2 * c
        jac = 6 * (n * (n - 1) / 2) * 40 * n            # one-sided Jacobi on the core
        qapply = 4 * c * c * (c * c) * 16               # Q times the kept singular vectors
        return qr + core + jac + qapply
    if stage == "bp_sweep":                             # two messages, 6 chi^4 complex MACs each
        return 2 * 6 * c ** 4 * 8
    if stage == "canonicalise":                         # 2 Cholesky, core, chi x chi Jacobi, 2 gauge maps
        return 8 * (2 * c ** 3 / 3.0 + c ** 3 + 2 * c ** 3) + 6 * (c * (c - 1) / 2) * 40 * c
    if stage == "gauge_apply":                          # three leg contractions of 2 chi^4 complex MACs
        return 3 * 2 * c ** 4 * 8
    return 0.0


def roofline_for(stage, prof, chi, precision):
    launches, tot_ms, items = prof[stage]
    avg_s = tot_ms / launches * 1e-3
    per_launch_items = items / launches
    by = algorithmic_bytes_per_item(stage, chi, precision) * per_launch_items
    fl = algorithmic_flops_per_item(stage, chi) * per_launch_items
    # FP64 arithmetic: the simple update and canonicalisation always; the rest in FP64 mode
    fp64 = precision == "fp64" or stage in ("simple_update", "canonicalise")
    alu_peak = FP64_VECTOR_PEAK_TFLOPS if fp64 else FP32_VECTOR_PEAK_TFLOPS
    t_mem = by / (HBM_PEAK_GBS * 1e9)
    t_alu = fl / (alu_peak * 1e12)
    if t_alu > t_mem:
        ach = fl / avg_s / 1e12
        return {"bound": "alu", "achieved": round(ach, 3), "peak": alu_peak, "unit": "TFLOP/s",
                "frac": round(ach / alu_peak, 5), "traffic": None, "kernel": stage,
                "avg_launch_ms": round(avg_s * 1e3, 5), "launches": launches,
                "alg_flops_per_launch": round(fl), "alg_bytes_per_launch": round(by),
                "hbm_gbs_at_alg_bytes": round(by / avg_s / 1e9, 2)}
    ach = by / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 5), "traffic": None, "kernel": stage,
            "avg_launch_ms": round(avg_s * 1e3, 5), "launches": launches,
            "alg_bytes_per_launch": round(by), "alg_flops_per_launch": round(fl)}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def _source_sha():
    from paper_2409_12240_amd.rocprof_summary import source_sha256
    return source_sha256()


def measured_traffic(stage, chi, precision, items_per_launch):
    """HBM bytes per launch of `stage` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE measurement, or None when there is none for this kernel and
    configuration or the kernel source has changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        sha = _source_sha()
    except (OSError, ValueError):
        return None
    hits = [r for r in rec.get("kernels", [])
            if (r.get("stage") == stage and r.get("chi") == chi and r.get("precision") == precision
                and r.get("items_per_launch") == items_per_launch and r.get("source_sha256") == sha)]
    if not hits:
        return None
    # a stage launch runs one of its main kernels (e.g. the BP variant for the
    # first class of a first sweep, or the general one) plus any companion
    # (the simple update's redo launch): the traffic per stage launch is the
    # call-weighted sum over the profiled run
    main_calls = sum(r.get("calls") or 0 for r in hits if not r.get("companion"))
    if main_calls <= 0 or any(r.get("calls") is None for r in hits):
        return None
    return round(sum(r["traffic_bytes_per_launch"] * r["calls"] for r in hits) / main_calls)


def measured_valu_busy(stage, chi, precision):
    """VALU issue time / kernel time of `stage` from the committed SQ counter
    pass (SQ_INSTS_VALU x 4 cycles over 1024 SIMDs at 2.4 GHz, against the
    rocprofv3 average duration), or None when the kernel source changed."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
        sha = _source_sha()
    except (OSError, ValueError):
        return None
    if not any(r.get("source_sha256") == sha for r in rec.get("kernels", [])):
        return None
    best = None
    for r in rec.get("sq", []):
        if (r.get("stage") == stage and r.get("valu_busy") is not None and r.get("chi", 4) == chi
                and r.get("precision", "mixed") == precision):
            if best is None or r["valu_issue_us"] > best["valu_issue_us"]:
                best = r
    return None if best is None else round(best["valu_busy"], 3)


def step_bytes(insts, chi, precision, sweeps_per_regauge, regauges_per_step=None):
    """Algorithmic HBM bytes of one Trotter step of every instance: per
    instance |E|(4G+6L) for the simple updates plus, per re-gauging,
    S n(G+6M) for the BP sweeps, 2nG for the gauge fix and |E|(2M+L) for
    the bond factorisations (S = measured sweeps per re-gauging; one
    re-gauging per colour class unless regauges_per_step is given)."""
    w = 8 if precision == "mixed" else 16
    G = 2 * chi ** 3 * w
    M = chi * chi * w
    L = 8 * chi
    tot = 0.0
    for inst in insts:
        n, m = inst.n, inst.n_edges
        C = int(inst.n_colours) if regauges_per_step is None else regauges_per_step
        tot += m * (4 * G + 6 * L) + C * (sweeps_per_regauge * n * (G + 6 * M) + 2 * n * G + m * (2 * M + L))
    return tot


def make_pool(gtqa, dev, insts, chi, precision, bp_tol, bp_max_sweeps, **opts):
    n_tot = sum(i.n for i in insts)
    pool = gtqa.Pool(chi=chi, precision=precision, max_vertices=n_tot,
                     max_edges=sum(i.n_edges for i in insts), max_slots=len(insts), device=dev,
                     bp_tol=bp_tol, bp_max_sweeps=bp_max_sweeps, **opts)
    slots = [pool.admit(i) for i in insts]
    if min(slots) < 0:
        raise RuntimeError("pool admission failed")
    return pool, slots


class Stepper:
    """A pool whose slots each follow the schedule at their own step index
    (k[s] steps done), so subsets of the slots can be timed in turn."""

    def __init__(self, torch, pool, slots, tz, tx):
        self.torch, self.pool, self.slots, self.tz, self.tx = torch, pool, list(slots), tz, tx
        self.k = {s: 0 for s in slots}

    def step(self, slots, n):
        for _ in range(n):
            ks = [self.k[s] for s in slots]
            self.pool.step(slots, self.tz[ks], self.tx[ks])
            for s in slots:
                self.k[s] += 1

    def timed(self, slots, n, edges_per_slot):
        """Time n steps of `slots` (synchronised on both sides); returns
        (seconds, gate-updates/s, k range, BP sweeps per re-gauging)."""
        before = [self.pool.bp_totals(s) for s in slots]
        k0 = min(self.k[s] for s in slots)
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        self.step(slots, n)
        self.torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        after = [self.pool.bp_totals(s) for s in slots]
        sw = sum(a[0] - b[0] for a, b in zip(after, before))
        rg = sum(a[1] - b[1] for a, b in zip(after, before))
        return secs, len(slots) * edges_per_slot * n / secs, (k0 + 1, max(self.k[s] for s in slots)), \
            sw / max(rg, 1)


def profile_every(K):
    """Stage timing in one step of every profile_every(K) of a K-step window:
    the events cost a step ~4 % when every launch carries them, so at most
    one step in eight is timed (at least ten steps of every window)."""
    return max(1, min(8, K // 10))


def time_pool(torch, gtqa, dev, insts, chi, precision, bp_tol, bp_max_sweeps, k0, K, tz, tx, read=0, **opts):
    """Untimed pre-roll to step k0, then K timed steps (k0+1 .. k0+K) with
    stage timing on in one step of every profile_every(K).  Returns (seconds,
    profile, sweeps per re-gauging, re-gaugings per slot and step, readouts
    of the first `read` slots)."""
    pool, slots = make_pool(gtqa, dev, insts, chi, precision, bp_tol, bp_max_sweeps, **opts)
    st = Stepper(torch, pool, slots, tz, tx)
    st.step(slots, k0)
    before = [pool.bp_totals(s) for s in slots]
    pool.profile(True)
    pool.profile_sample(profile_every(K))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.step(slots, K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pool.profile_read()
    after = [pool.bp_totals(s) for s in slots]
    sweeps = sum(a[0] - b[0] for a, b in zip(after, before))
    regauges = sum(a[1] - b[1] for a, b in zip(after, before))
    outs = [pool.readout(s) for s in slots[:read]]
    pool.close()
    return t1 - t0, prof, sweeps / max(regauges, 1), regauges / (len(slots) * K), outs


def comparison_legs(torch, gtqa, dev, insts, chi, l0, L, tz, tx, batches, bp_max_sweeps):
    """Batched vs plain, precision vs BP tolerance, batch size: for each
    precision one pool of every instance, pre-rolled (untimed, at its own
    tolerance: 1e-6 mixed, 1e-10 FP64) to step l0; then L timed steps for
    the first B slots, for each B in `batches` (largest first, every slot at
    its own step index), and finally L steps of all slots at the other
    tolerance."""
    edges = insts[0].n_edges
    out = {"window_start_k": l0 + 1, "steps_per_window": L, "legs": []}
    for precision, tol, other in (("mixed", 1e-6, 1e-10), ("fp64", 1e-10, 1e-6)):
        pool, slots = make_pool(gtqa, dev, insts, chi, precision, tol, bp_max_sweeps)
        st = Stepper(torch, pool, slots, tz, tx)
        st.step(slots, l0)
        for B in sorted(batches, reverse=True):
            secs, rate, kr, sw = st.timed(slots[:B], L, edges)
            out["legs"].append({"precision": precision, "bp_tol": tol, "batch": B,
                                "gate_updates_per_s": round(rate, 1), "ms_per_step": round(secs / L * 1e3, 4),
                                "k": list(kr), "bp_sweeps_per_regauge": round(sw, 3)})
        pool.set_bp(other, bp_max_sweeps)
        B = max(batches)
        secs, rate, kr, sw = st.timed(slots[:B], L, edges)
        out["legs"].append({"precision": precision, "bp_tol": other, "batch": B,
                            "gate_updates_per_s": round(rate, 1), "ms_per_step": round(secs / L * 1e3, 4),
                            "k": list(kr), "bp_sweeps_per_regauge": round(sw, 3)})
        pool.close()
    return out


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model or platform.processor() or platform.machine(),
            "nproc": usable, "os_cpu_count": os.cpu_count()}


MID_STATE = os.path.join(ROOT, "tests", "golden", "anneal_n1000_s1000_chi4_state_k1000.npz")

CPU_SAMPLE_CODE = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, {root!r})
from synthetic import random_regular_instance, schedule_angles
from oracle import gtqa as G
state_file = {state!r}
seed = 1000 if state_file else 2000
inst = random_regular_instance(seed, {n})
st = G.init_state(inst, G.Options(chi={chi}, bp_tol={tol}, bp_max_sweeps={maxs}))
k = 0
if state_file:
    d = np.load(state_file)
    dims = [int(x) for x in d["dims"]]
    for a in range(inst.n):
        legs = [dims[e] for e in st.inc[a]]
        st.gamma[a] = np.array(d["gamma"][a][(slice(None),) + tuple(slice(0, x) for x in legs)])
    for e in range(inst.n_edges):
        st.lam[e] = np.array(d["lam"][e][:dims[e]])
    k = int(d["k"])
tz, tx = schedule_angles({T}, {dt})
k_first = k + 1
t0 = time.perf_counter(); sweeps = []
while k < len(tz):
    s = G.trotter_step(st, tz[k], tx[k]); sweeps += s.sweeps; k += 1
    if time.perf_counter() - t0 > {budget} or k - k_first + 1 >= {kmax}:
        break
dt_ = time.perf_counter() - t0
print(json.dumps({{"steps": k - k_first + 1, "k_first": k_first, "k_last": k, "seed": seed,
                   "seconds": dt_, "gate_updates": (k - k_first + 1) * inst.n_edges, "sweeps": sweeps}}))
"""


def cpu_baseline(args):
    env = dict(os.environ)
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "NUMEXPR_NUM_THREADS"):
        env[v] = "1"
    state = MID_STATE if (args.n == 1000 and args.chi == 4 and os.path.exists(MID_STATE)) else ""
    code = CPU_SAMPLE_CODE.format(root=ROOT, state=state, n=args.n, chi=args.chi, tol=1e-10, maxs=50,
                                  T=args.T, dt=args.dt, kmax=args.cpu_max_steps, budget=args.cpu_seconds)
    out = subprocess.run([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE,
                         stderr=subprocess.PIPE, text=True, timeout=900)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    r = json.loads(out.stdout.strip().splitlines()[-1])
    rate = r["gate_updates"] / r["seconds"]
    where = ("from the oracle's own network after step 1000 (tests/golden), i.e. mid-anneal"
             if state else "from |+>^N")
    cpu = host_cpu()
    return {"value": rate, "unit": "gate-updates/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu["cpu_model"], "nproc": cpu["nproc"],
            "sample": (f"oracle (complex128 NumPy, 1 thread, BP 1e-10/50) on a random 3-regular "
                       f"instance n={args.n} (seed {r['seed']}), chi={args.chi}, steps "
                       f"k={r['k_first']}..{r['k_last']} of the T={args.T:g}, dt={args.dt:g} schedule "
                       f"{where}, {r['seconds']:.1f} s, BP sweeps per re-gauging "
                       f"{min(r['sweeps'])}..{max(r['sweeps'])} (mean {sum(r['sweeps'])/len(r['sweeps']):.2f})")}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1990)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--chi", type=int, default=4)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--T", type=float, default=100.0)
    ap.add_argument("--dt", type=float, default=0.05)
    ap.add_argument("--bp-tol", type=float, default=None)
    ap.add_argument("--bp-max-sweeps", type=int, default=50)
    ap.add_argument("--leg-steps", type=int, default=40,
                    help="timed steps per comparison leg (mid-anneal window; 0: skip the legs)")
    ap.add_argument("--leg-batches", type=str, default="1,8,32,128,256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-max-steps", type=int, default=20)
    ap.add_argument("--detail", action="store_true", help="per-stage breakdown on stderr")
    ap.add_argument("--serve-jobs", type=int, default=8,
                    help="jobs per arrival rate in the serving sweep (0: skip)")
    ap.add_argument("--serve-chis", type=str, default="4,8,16")
    ap.add_argument("--chi16-batch", type=int, default=16,
                    help="instances in the chi=16 leg (0: skip)")
    ap.add_argument("--chi16-steps", type=int, default=10)
    ap.add_argument("--chi16-window-start", type=int, default=200)
    ap.add_argument("--mixed-chi-batch", type=int, default=256,
                    help="instances in the mixed-chi batch leg (chi 4 / 8 alternating; 0: skip)")
    ap.add_argument("--adaptive-residual-max", type=float, default=1e-3,
                    help="also time adaptive re-gauging with this threshold on R (<= 0: skip)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this size (for HBM counter scaling)")
    ap.add_argument("--only-headline", action="store_true",
                    help="time the headline window only (for profiling runs)")
    ap.add_argument("--window-start", type=int, default=None,
                    help="timed window starts after step k0 (default: centred in the anneal)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(instances shard across GPUs with no exchange; see the design notes)"}))
        sys.exit(2)

    import torch

    from paper_2409_12240_amd import gtqa
    from synthetic import random_regular_instance, schedule_angles

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = gtqa.TorchDevice()
    if args.copy_calibration_mib > 0:
        src = torch.empty(args.copy_calibration_mib << 20, dtype=torch.uint8, device="cuda")
        src.fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tz, tx = schedule_angles(args.T, args.dt)
    n_sched = tz.size
    W, K = args.warmup, args.steps
    if W + K > n_sched:
        raise SystemExit("warmup + steps exceed the schedule length")
    # the timed window sits in the middle of the anneal (the whole anneal when
    # K fills it): an untimed pre-roll of k0 steps, whose last W are the warm-up
    k0 = max(W, (n_sched - K) // 2) if args.window_start is None else max(W, args.window_start)
    if k0 + K > n_sched:
        raise SystemExit("the timed window runs past the end of the schedule")
    bp_tol = args.bp_tol if args.bp_tol is not None else (1e-6 if args.precision == "mixed" else 1e-10)
    insts = [random_regular_instance(2000 + i, args.n) for i in range(args.batch)]
    n_edges = insts[0].n_edges

    for inst in insts:
        inst.n_colours = int(gtqa.gtqa_colour_edges(inst.n, inst.edges).max()) + 1
    n_read = min(4, args.batch)
    secs, prof, mean_sweeps, _, ref_out = time_pool(torch, gtqa, dev, insts, args.chi, args.precision, bp_tol,
                                                    args.bp_max_sweeps, k0, K, tz, tx, read=n_read)
    value = args.batch * n_edges * K / secs
    log(f"headline: {value / 1e6:.2f} M gate-updates/s ({secs / K * 1e3:.3f} ms per step)")
    bstep = step_bytes(insts, args.chi, args.precision, mean_sweeps)
    step_roofline = {"bound": "hbm", "alg_bytes_per_step": round(bstep),
                     "achieved": round(bstep * K / secs / 1e9, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(bstep * K / secs / 1e9 / HBM_PEAK_GBS, 5),
                     "sweeps_per_regauge": round(mean_sweeps, 4)}

    # dominant kernel by total event time over the timed region
    stage_ms = {k: v[1] for k, v in prof.items() if v[0] > 0}
    dom = max(stage_ms, key=stage_ms.get)
    roofline = roofline_for(dom, prof, args.chi, args.precision)
    roofline["traffic"] = measured_traffic(dom, args.chi, args.precision, round(prof[dom][2] / prof[dom][0]))
    roofline["valu_issue_busy"] = measured_valu_busy(dom, args.chi, args.precision)
    kernels = {st: roofline_for(st, prof, args.chi, args.precision)
               for st in ("simple_update", "bp_sweep", "canonicalise", "gauge_apply") if st in stage_ms}
    for st, r in kernels.items():
        r["traffic"] = measured_traffic(st, args.chi, args.precision, round(prof[st][2] / prof[st][0]))
        r["valu_issue_busy"] = measured_valu_busy(st, args.chi, args.precision)

    adaptive = None
    if args.adaptive_residual_max > 0 and not args.only_headline:
        import numpy as np
        asecs, aprof, _, a_rps, a_out = time_pool(torch, gtqa, dev, insts, args.chi, args.precision, bp_tol,
                                                  args.bp_max_sweeps, k0, K, tz, tx, read=n_read,
                                                  regauge="adaptive", residual_max=args.adaptive_residual_max)
        adaptive = {"residual_max": args.adaptive_residual_max,
                    "gate_updates_per_s": round(args.batch * n_edges * K / asecs, 1),
                    "ms_per_step": round(asecs / K * 1e3, 4),
                    "regauges_per_step": round(a_rps, 4),
                    "stage_ms": {k: round(v[1], 3) for k, v in aprof.items() if v[0] > 0},
                    "max_abs_dz_vs_every_class": float(max(np.max(np.abs(a["z"] - r["z"]))
                                                           for a, r in zip(a_out, ref_out))),
                    "bits_differing_vs_every_class": int(sum(int(np.sum(a["x"] != r["x"]))
                                                             for a, r in zip(a_out, ref_out))),
                    "compared_instances": n_read}
        log(f"adaptive re-gauging: {adaptive['gate_updates_per_s'] / 1e6:.2f} M gate-updates/s")

    legs = None
    plain = None
    plain_sweeps = None
    if args.leg_steps > 0 and not args.only_headline:
        batches = sorted({min(int(b), args.batch) for b in args.leg_batches.split(",")})
        L = args.leg_steps
        l0 = (n_sched - (len(batches) + 1) * L) // 2
        legs = comparison_legs(torch, gtqa, dev, insts, args.chi, l0, L, tz, tx, batches, args.bp_max_sweeps)
        for leg in legs["legs"]:
            if leg["precision"] == "fp64" and leg["bp_tol"] == 1e-10 and leg["batch"] == 1:
                plain, plain_sweeps = leg["gate_updates_per_s"], leg["bp_sweeps_per_regauge"]
        log(f"comparison legs done ({len(legs['legs'])} windows)")

    mixed_chi = None
    if args.mixed_chi_batch > 0 and not args.only_headline:
        from paper_2409_12240_amd.batch import MixedChiBatch, mixed_chi_instances, summary
        minsts, mchis = mixed_chi_instances(count=args.mixed_chi_batch)
        mixed_chi = {"workload": f"{args.mixed_chi_batch} random 3-regular instances, n = 2 U{{25..250}}, "
                                 "chi 4 (even index) / 8 (odd), T=20 dt=0.05 (400 steps), whole anneal, "
                                 "one pool per chi on its own stream, run concurrently"}
        for prec in ("mixed", "fp64"):
            mb = MixedChiBatch(minsts, mchis, precision=prec)
            _, mwall, mwalls = mb.anneal(20.0, 0.05, read=False)
            mixed_chi[prec] = summary(minsts, mchis, mwall, mwalls, 400, mb.bp_sweeps)
            log(f"mixed-chi batch {prec}: {mwall:.2f} s")

    wide = None
    if args.chi16_batch > 0 and not args.only_headline:
        # the chi=16 path (MFMA contractions): B resident n=1000 instances,
        # pre-rolled to a window where every bond has reached 16
        winsts = insts[:min(args.chi16_batch, len(insts))]
        wide = {"workload": f"{len(winsts)} random 3-regular instances n={args.n} chi=16, T={args.T:g} "
                            f"dt={args.dt:g}, timed steps k={args.chi16_window_start + 1}.."
                            f"{args.chi16_window_start + args.chi16_steps} after an untimed pre-roll"}
        for prec, tol in (("mixed", 1e-6), ("fp64", 1e-10)):
            wsecs, wprof, wsw, _, _ = time_pool(torch, gtqa, dev, winsts, 16, prec, tol, args.bp_max_sweeps,
                                                args.chi16_window_start, args.chi16_steps, tz, tx)
            wide[prec] = {"bp_tol": tol,
                          "gate_updates_per_s": round(len(winsts) * n_edges * args.chi16_steps / wsecs, 1),
                          "ms_per_step": round(wsecs / args.chi16_steps * 1e3, 4),
                          "bp_sweeps_per_regauge": round(wsw, 4),
                          "stage_ms": {k: round(v[1], 3) for k, v in wprof.items() if v[0] > 0},
                          "kernel_rooflines": {st: roofline_for(st, wprof, 16, prec)
                                               for st in ("simple_update", "bp_sweep", "canonicalise", "gauge_apply")
                                               if wprof.get(st, (0,))[0] > 0}}
            for st, r in wide[prec]["kernel_rooflines"].items():
                r["traffic"] = measured_traffic(st, 16, prec, round(wprof[st][2] / wprof[st][0]))
            log(f"chi=16 {prec}: {wide[prec]['gate_updates_per_s'] / 1e6:.3f} M gate-updates/s "
                f"({wide[prec]['ms_per_step']:.2f} ms per step)")

    serving = None
    if args.serve_jobs > 0 and not args.only_headline:
        from paper_2409_12240_amd.serve import rate_sweep
        chis = tuple(int(c) for c in args.serve_chis.split(","))
        serving = rate_sweep(jobs_per_rate=args.serve_jobs, chis=chis, precision=args.precision, progress=log)
        serving["workload"] = ("Poisson arrivals at rho x measured capacity; n=2*U{50..1000}, chi uniform "
                               "over chis (chi=16 on the MFMA path), steps U{200..2000}, dt=0.05; "
                               "HBM-footprint admission")

    cpu = None if (args.no_cpu_baseline or args.only_headline) else cpu_baseline(args)
    if cpu is not None:
        log("cpu baseline done")

    if args.detail:
        tot = sum(stage_ms.values())
        for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1]):
            if v[0]:
                print(f"  {k:14s} launches {v[0]:6d}  total {v[1]:9.2f} ms  ({100*v[1]/max(tot,1e-9):5.1f}%)"
                      f"  avg {v[1]/v[0]*1e3:8.1f} us  items/launch {v[2]/v[0]:.0f}", file=sys.stderr)
        ev = profile_every(K)
        print(f"  wall {secs*1e3:.1f} ms for {K} steps; stage sum {tot:.1f} ms over the "
              f"{(K + ev - 1) // ev} timed steps (one in {ev})", file=sys.stderr)

    dtype = "c64+f64" if args.precision == "mixed" else "c128"
    line = {
        "metric": "Trotter gate-updates/s at n=1000 chi=4 (batched vs plain); p50/p99 anneal latency",
        "value": round(value, 1),
        "unit": "gate-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(secs / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"batched GTQA Trotter steps, {args.batch} random 3-regular instances "
                               f"n={args.n} chi={args.chi}, T={args.T:g} dt={args.dt:g}, timed steps "
                               f"k={k0+1}..{k0+K} of {n_sched} after an untimed pre-roll of k=1..{k0}",
                   "batch": args.batch, "n": args.n, "chi": args.chi, "precision": args.precision,
                   "bp_tol": bp_tol, "timed_k": [k0 + 1, k0 + K], "parallelism": "single-gpu"},
        "plain_fp64_gate_updates_per_s": plain,
        "plain_fp64_bp_sweeps_per_regauge": plain_sweeps,
        "stage_ms": {k: round(v, 3) for k, v in stage_ms.items()},
        "stage_timed_steps": {"every": profile_every(K), "count": (K + profile_every(K) - 1) // profile_every(K)},
        "bp_sweeps_per_regauge": round(mean_sweeps, 4),
        "comparison": legs,
        "mixed_chi_batch": mixed_chi,
        "chi16": wide,
        "serving": serving,
        "roofline": roofline,
        "kernel_rooflines": kernels,
        "step_roofline": step_roofline,
        "adaptive_regauge": adaptive,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
