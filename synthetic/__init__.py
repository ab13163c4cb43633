"""Seeded synthetic inputs for the GTQA Trotter-step engine.

This package generates problem instances only: random simple 3-regular graphs
(and small trees / hand-made graphs for tests) with couplings J_ab and fields
h_a.  It contains none of the annealing method's arithmetic, so both the CPU
oracle and the GPU path may use it to obtain identical inputs.
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
