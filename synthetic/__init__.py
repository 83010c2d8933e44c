"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package only draws random numbers and lays them out as canonical FP32 arrays.  It holds
none of the validated computation: no forward kinematics of a configuration, no clearance and
no collision test.  The robot and scene layouts follow the workloads described for the
method's evaluation (7-, 8- and 14-DoF arms; shelf, tabletop and cluttered scenes), drawn from
one root seed so every consumer sees bit-identical inputs.
"""
from .robots import (chain_robot, bimanual_robot, lift_arm_robot, robot_summary, link_parents,
                     candidate_pairs)
from .scenes import (cube_scene, shelf_scene, point_cloud_scene, random_scene,
                     empty_scene, scene_summary)
from .workloads import (ROOT_SEED, rng, uniform_states, uniform_edges, trajectories,
                        workload, pack_edge_sets)

__all__ = [
    "chain_robot", "bimanual_robot", "lift_arm_robot", "robot_summary", "link_parents", "candidate_pairs",
    "cube_scene", "shelf_scene", "point_cloud_scene", "random_scene", "empty_scene",
    "scene_summary", "ROOT_SEED", "rng", "uniform_states", "uniform_edges", "trajectories",
    "workload", "pack_edge_sets",
]
