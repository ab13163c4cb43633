"""Batches of instances with different bond dimensions (mixed chi).

The kernels are specialised on chi (register and LDS layouts differ between
chi = 4 and chi = 8), so a batch whose instances differ in chi is split into
one pool per chi.  Each pool lives on its own HIP stream and is advanced by
its own host thread, so the per-chi launch sequences (one launch per kernel
stage covering every instance of that chi) run concurrently on the device.
Every instance's arithmetic is independent of the other instances in its
pool, so a result does not depend on the batch it ran in.

This module only marshals: every step runs in libgtqa through its pool calls.
"""

from __future__ import annotations

import threading
import time

import numpy as np

from . import gtqa


class MixedChiBatch:
    """Runs the first-order anneal (App. F) of many instances with per-instance
    chi: one pool per chi, each stepped by its own thread on its own stream."""

    def __init__(self, instances, chis, precision="mixed", device_factory=None, **opts):
        if len(instances) != len(chis):
            raise ValueError("one chi per instance")
        self.instances = list(instances)
        self.chis = [int(c) for c in chis]
        self.precision = precision
        self.opts = opts
        self.device_factory = device_factory or (lambda: gtqa.TorchDevice(stream="own"))

    def groups(self):
        out = {}
        for i, c in enumerate(self.chis):
            out.setdefault(c, []).append(i)
        return out

    def anneal(self, T: float, dt: float, read: bool = True, timeout_s: float = 1800.0):
        """Whole anneal of every instance (K = round(T/dt) steps, step k with
        theta_z = dt k / K, theta_x = dt (K - k) / K).  Returns (readouts in
        instance order or None, wall seconds of the stepping, per-chi wall
        seconds)."""
        from synthetic import schedule_angles
        tz, tx = schedule_angles(T, dt)
        results = [None] * len(self.instances)
        walls = {}
        self.bp_sweeps = {}
        spans = []
        errors = []
        start = threading.Barrier(len(self.groups()) + 1)

        def run(chi, idx):
            try:
                dev = self.device_factory()
                insts = [self.instances[i] for i in idx]
                pool = gtqa.Pool(chi=chi, precision=self.precision, max_vertices=sum(x.n for x in insts),
                                 max_edges=sum(x.n_edges for x in insts), max_slots=len(insts), device=dev,
                                 **self.opts)
                try:
                    slots = [pool.admit(x) for x in insts]
                    if min(slots) < 0:
                        raise RuntimeError("pool admission failed")
                    dev.torch.cuda.synchronize()
                    start.wait()
                    t0 = time.perf_counter()
                    for k in range(tz.size):
                        pool.step(slots, tz[k], tx[k])
                    dev.stream.synchronize()
                    t1 = time.perf_counter()
                    walls[chi] = t1 - t0
                    spans.append((t0, t1))
                    tot = [pool.bp_totals(sl) for sl in slots]
                    self.bp_sweeps[chi] = (sum(a for a, _ in tot) / max(1, sum(b for _, b in tot)),
                                           max(a / max(1, b) for a, b in tot))
                    if read:
                        for i, s in zip(idx, slots):
                            results[i] = pool.readout(s)
                finally:
                    pool.close()
            except BaseException as exc:
                errors.append(exc)
                try:
                    start.abort()
                except threading.BrokenBarrierError:
                    pass

        threads = [threading.Thread(target=run, args=(c, idx), daemon=True) for c, idx in self.groups().items()]
        for th in threads:
            th.start()
        try:
            start.wait()
        except threading.BrokenBarrierError:
            pass
        for th in threads:
            th.join(timeout=timeout_s)
        if errors:
            raise errors[0]
        if any(th.is_alive() for th in threads):
            raise TimeoutError("mixed-chi batch did not finish")
        # from the first pool's first step to the last pool's last step
        wall = max(b for _, b in spans) - min(a for a, _ in spans)
        return (results if read else None), wall, walls


def mixed_chi_instances(count=256, seed0=2000, n_half_range=(25, 250)):
    """The mixed-chi batch workload: instance i is a random 3-regular graph on
    n = 2 U{25..250} vertices (drawn from SplitMix64(seed0 + 7919 i)), seed
    seed0 + i, chi = 4 for even i and 8 for odd i."""
    from synthetic import SplitMix64, random_regular_instance
    insts, chis = [], []
    for i in range(count):
        r = SplitMix64(seed0 + 7919 * i)
        n = 2 * (n_half_range[0] + r.bounded(n_half_range[1] - n_half_range[0] + 1))
        insts.append(random_regular_instance(seed0 + i, n))
        chis.append(4 if i % 2 == 0 else 8)
    return insts, chis


def gate_updates(instances, steps: int) -> int:
    return int(sum(x.n_edges for x in instances)) * int(steps)


def summary(instances, chis, wall, walls, steps, bp_sweeps=None):
    n = np.array([x.n for x in instances])
    out = {"instances": len(instances), "chi_counts": {str(c): int(sum(1 for x in chis if x == c)) for c in set(chis)},
           "n_min": int(n.min()), "n_max": int(n.max()), "n_mean": round(float(n.mean()), 1),
           "steps": steps, "wall_s": round(wall, 4),
           "per_chi_wall_s": {str(c): round(w, 4) for c, w in walls.items()},
           "gate_updates_per_s": round(gate_updates(instances, steps) / wall, 1)}
    if bp_sweeps:
        out["bp_sweeps_per_regauge"] = {str(c): {"mean": round(m, 3), "max_instance_mean": round(x, 3)}
                                        for c, (m, x) in bp_sweeps.items()}
    return out
