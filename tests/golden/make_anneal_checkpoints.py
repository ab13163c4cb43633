"""Write oracle checkpoint fixtures for whole anneals (App. F, Sec. III.A).

Calls only the oracle (`oracle.gtqa.anneal`) and the seeded instance
generator.  For one random 3-regular instance it runs the first-order anneal
with re-gauging after every colour class and BP to dist/|E| < bp_tol (at most
bp_max_sweeps sweeps), and stores at each checkpoint step k the readout
<Z_a>, the rounded string and E(x); for every step the BP sweep counts of each
re-gauging, the final dist/|E|, the step's log-fidelity sum and largest
truncation error.  The file is rewritten after every checkpoint, so a run that
is stopped early still leaves every checkpoint it reached.

`--relabel SEED` runs the same instance with its vertices renamed by a
seeded permutation and with the original colouring carried over, so that the
gates, their order and the BP schedule are the same operations: only the leg
order of each tensor, hence the order of every sum, changes.  The readout is
mapped back to the original vertex names.  Two such runs measure how far two
correct implementations of the same arithmetic drift apart (the sensitivity
floor of the comparison).

Example (n = 1000, T = 100, dt = 0.05, chi = 4, one core):
  OMP_NUM_THREADS=1 python tests/golden/make_anneal_checkpoints.py \
      --n 1000 --seed 1000 --chi 4 --T 100 --dt 0.05 \
      --checkpoints 1,10,100,250,500,1000,1500,2000 \
      --out tests/golden/anneal_n1000_s1000_chi4.json
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

from oracle import gtqa as O                       # noqa: E402
from oracle.colouring import misra_gries          # noqa: E402
from synthetic import SplitMix64, Instance, random_regular_instance  # noqa: E402


def relabelled(inst: Instance, colour: np.ndarray, seed: int):
    """The same graph and couplings with vertex a renamed perm[a] (a seeded
    Fisher-Yates permutation); edges re-sorted with u < v.  Returns the new
    instance, its colouring (each edge keeps its colour) and perm."""
    rng = SplitMix64(seed)
    perm = list(range(inst.n))
    for i in range(inst.n - 1, 0, -1):
        j = rng.bounded(i + 1)
        perm[i], perm[j] = perm[j], perm[i]
    perm = np.asarray(perm, dtype=np.int64)
    rows = []
    for e in range(inst.n_edges):
        u, v = perm[int(inst.edges[e, 0])], perm[int(inst.edges[e, 1])]
        rows.append((min(u, v), max(u, v), e))
    rows.sort()
    old = [r[2] for r in rows]
    edges = np.array([[r[0], r[1]] for r in rows], dtype=np.int32)
    J = np.asarray(inst.J)[old].copy()
    h = np.zeros(inst.n)
    h[perm] = inst.h
    col = np.asarray(colour)[old].copy()
    return Instance(n=inst.n, edges=edges, J=J, h=h, seed=inst.seed,
                    meta={"kind": "relabelled", "perm_seed": seed}), col, perm


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--seed", type=int, required=True)
    ap.add_argument("--chi", type=int, default=4)
    ap.add_argument("--T", type=float, required=True)
    ap.add_argument("--dt", type=float, required=True)
    ap.add_argument("--bp-tol", type=float, default=1e-10)
    ap.add_argument("--bp-max-sweeps", type=int, default=50)
    ap.add_argument("--checkpoints", type=str, required=True)
    ap.add_argument("--relabel", type=int, default=None)
    ap.add_argument("--out", type=str, required=True)
    ap.add_argument("--save-state", type=str, default="",
                    help="checkpoint steps at which the whole network is also saved "
                         "(<out stem>_state_k<k>.npz)")
    a = ap.parse_args(argv)

    inst = random_regular_instance(a.seed, a.n)
    colour = misra_gries(inst.n, inst.edges)
    perm = np.arange(inst.n)
    run_inst, run_col = inst, colour
    if a.relabel is not None:
        run_inst, run_col, perm = relabelled(inst, colour, a.relabel)
    cps = sorted(int(x) for x in a.checkpoints.split(","))
    state_ks = {int(x) for x in a.save_state.split(",") if x}
    if a.relabel is not None and state_ks:
        raise SystemExit("--save-state is for runs without --relabel")
    opts = O.Options(chi=a.chi, bp_tol=a.bp_tol, bp_max_sweeps=a.bp_max_sweeps)
    t0 = time.time()
    meta = {
        "what": "oracle anneal checkpoints (App. F first-order circuit, linear schedule, "
                "re-gauging after every colour class)",
        "script": "tests/golden/make_anneal_checkpoints.py",
        "argv": sys.argv[1:] if argv is None else list(argv),
        "n": a.n, "seed": a.seed, "chi": a.chi, "T": a.T, "dt": a.dt,
        "bp_tol": a.bp_tol, "bp_max_sweeps": a.bp_max_sweeps,
        "relabel_seed": a.relabel, "n_colours": int(np.max(colour)) + 1,
        "host": platform.node(), "cpu": platform.processor() or platform.machine(),
    }

    def save(k, out):
        stats = out["stats"]
        doc = dict(meta)
        doc["wall_s"] = time.time() - t0
        doc["steps_done"] = len(stats)
        doc["sweeps"] = [list(map(int, s.sweeps)) for s in stats]
        doc["dists"] = [[float(d) for d in s.dists] for s in stats]
        doc["log_fidelity"] = [float(s.log_fidelity) for s in stats]
        doc["max_eps"] = [float(s.max_eps) for s in stats]
        doc["checkpoints"] = {}
        for kk, c in sorted(out["checkpoints"].items()):
            z = np.asarray(c["z"])[perm]          # back to the original vertex names
            x = np.asarray(c["x"])[perm]
            doc["checkpoints"][str(kk)] = {
                "z": [float(v) for v in z],
                "x": "".join("+" if v > 0 else "-" for v in x),
                "E": float(c["E"]),
                "undecided_1e-9": int(np.sum(np.abs(z) <= 2e-9)),
            }
        tmp = a.out + ".tmp"
        with open(tmp, "w") as f:
            json.dump(doc, f, separators=(",", ":"))
        os.replace(tmp, a.out)
        print(f"k={k} saved after {doc['wall_s']:.0f} s", flush=True)

    def save_all(k, out, state):
        save(k, out)
        if k in state_ks:
            save_network(state, a.out[:-len(".json")] + f"_state_k{k}.npz", k)

    O.anneal(run_inst, a.T, a.dt, opts, colour=run_col, checkpoints=cps, on_checkpoint=save_all)


def save_network(state, path: str, k: int) -> None:
    """The network after step k, zero-padded to chi: gamma [n][2][chi][chi][chi]
    (legs in ascending incident-edge order), lam [E][chi], bond dims [E]."""
    chi = state.opts.chi
    g = np.zeros((state.n, 2, chi, chi, chi), dtype=np.complex128)
    for a_ in range(state.n):
        G = state.gamma[a_]
        G = G.reshape(G.shape + (1,) * (4 - G.ndim))     # a missing leg uses index 0
        g[a_][tuple(slice(0, d) for d in G.shape)] = G
    lam = np.zeros((state.n_edges, chi))
    dims = np.zeros(state.n_edges, dtype=np.int32)
    for e in range(state.n_edges):
        lam[e, :state.lam[e].size] = state.lam[e]
        dims[e] = state.lam[e].size
    np.savez_compressed(path, gamma=g, lam=lam, dims=dims, k=np.int64(k))


if __name__ == "__main__":
    main()
