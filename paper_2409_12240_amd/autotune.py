"""Launch autotuner for libgtqa on the GPU it runs on.

Picks the process-wide launch configuration (gtqa_set_tuning) by timing:
  * su_edges_per_wave_chi4: 2 or 4 edges of the chi=4 simple update per
    64-lane wavefront (32 or 16 lanes per edge);
  * xcd_contiguous: work-groups reordered so each of the 8 XCDs takes a
    contiguous item range (its L2 then holds one instance's lambdas, messages
    and gauge maps), or the dispatcher's round-robin order;
  * canon_lanes_chi4: Alg. 2 at chi=4 with 4 lanes per edge (one per column
    of the bond core, 16 edges per wavefront) or 8 (8 edges per wavefront).
Every combination runs the same batched Trotter steps (a pool of random
3-regular instances advanced past the start of the anneal, where the bonds
have reached chi) with per-stage event timing; the combination with the least
total kernel time wins.  The table is written next to the library and applied
by the binding when it loads.

    python -m paper_2409_12240_amd.autotune [--batch 64] [--steps 8]
"""

from __future__ import annotations

import argparse
import itertools
import json
import os
import sys
import time

from . import gtqa

CANDIDATES = {"su_edges_per_wave_chi4": (2, 4), "xcd_contiguous": (0, 1), "canon_lanes_chi4": (4, 8)}


def tune(batch=64, n=1000, chi=4, precision="mixed", warm=200, steps=8, repeats=2, seed0=5000,
         out=gtqa.TUNING_FILE, verbose=True):
    import torch

    from synthetic import random_regular_instance, schedule_angles

    dev = gtqa.TorchDevice()
    insts = [random_regular_instance(seed0 + i, n) for i in range(batch)]
    tz, tx = schedule_angles(100.0, 0.05)
    # stage timing is on throughout, so every launch is direct (no graphs)
    pool = gtqa.Pool(chi=chi, precision=precision, max_vertices=n * batch, max_slots=batch, device=dev,
                     launch="direct")
    slots = [pool.admit(i) for i in insts]
    k = 0
    for _ in range(warm):
        pool.step(slots, tz[k], tx[k])
        k += 1
    torch.cuda.synchronize()
    names = list(CANDIDATES)
    trials = []
    for rep in range(repeats):
        for combo in itertools.product(*(CANDIDATES[m] for m in names)):
            cfg = dict(zip(names, combo))
            for m, v in cfg.items():
                gtqa.set_tuning(m, v)
            pool.profile(True)
            t0 = time.perf_counter()
            for _ in range(steps):
                pool.step(slots, tz[k], tx[k])
                k += 1
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            prof = pool.profile_read()
            pool.profile(False)
            kernel_ms = sum(v[1] for v in prof.values())
            trials.append({"config": cfg, "repeat": rep, "kernel_ms_per_step": kernel_ms / steps,
                           "wall_ms_per_step": 1e3 * wall / steps,
                           "stage_ms_per_step": {s: v[1] / steps for s, v in prof.items() if v[0]}})
            if verbose:
                print(json.dumps(trials[-1]), flush=True)
    pool.close()
    best = {}
    for t in trials:
        key = json.dumps(t["config"], sort_keys=True)
        best.setdefault(key, []).append(t["kernel_ms_per_step"])
    ranked = sorted(best.items(), key=lambda kv: min(kv[1]))
    choice = json.loads(ranked[0][0])
    for m, v in choice.items():
        gtqa.set_tuning(m, v)
    table = {"device": torch.cuda.get_device_name(0), "arch": "gfx950",
             "workload": {"batch": batch, "n": n, "chi": chi, "precision": precision,
                          "steps_after_warmup": warm, "timed_steps": steps, "repeats": repeats},
             "criterion": "least kernel time per Trotter step (best of the repeats)",
             "trials": trials, "choice": choice}
    if out:
        tmp = out + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(table, fh, indent=1)
        os.replace(tmp, out)
    return table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--warm", type=int, default=200)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--repeats", type=int, default=2)
    ap.add_argument("--out", default=gtqa.TUNING_FILE)
    a = ap.parse_args(argv)
    table = tune(batch=a.batch, n=a.n, warm=a.warm, steps=a.steps, repeats=a.repeats, out=a.out)
    print(json.dumps({"choice": table["choice"], "written": a.out}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
