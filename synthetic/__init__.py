"""Seeded synthetic inputs for the GTQA Trotter-step engine.

This package generates the inputs both the CPU oracle and the GPU path take:
random simple 3-regular graphs (and small trees / hand-made graphs for
tests) with couplings J_ab and fields h_a; the random numbers a run draws
(entries of Alg. 1's random start messages, by counter); and the angle
sequences of the product formulas (the time discretisation of the linear
schedule: first order as in App. F, symmetric second order, randomised
order).  The angle sequences are the only part of the method here; both
sides receive them as arguments, and neither side's tensor-network
arithmetic is shared.
"""

from .instances import (  # noqa: F401
    SplitMix64,
    Instance,
    random_regular_instance,
    random_tree_instance,
    instance_from_edges,
    grid_coupling,
    splitmix64_at,
    random_message_entries,
    schedule_angles,
    schedule_angles_second_order,
    schedule_angles_randomised,
)
