"""Seeded synthetic workloads shared, as data only, by the FP64 oracle and the HIP path.

This package holds model descriptions (tree topology, joint axes, masses,
inertias, contact spheres, gains) and seeded generators for initial states and
MLP weights.  It holds none of the simulation arithmetic: no kinematics, no
dynamics, no rewards.  Everything it returns is plain numpy data.
"""
from .models import (FREE, HINGE, SLIDE, cartpole, ant, humanoid, mtu_humanoid, model_by_name,
                     pendulum, free_body, sliding_block, chain, muscle_arm,
                     with_termination)
from .inputs import initial_states, mlp_params, workload, WORKLOADS

__all__ = ["FREE", "HINGE", "SLIDE", "cartpole", "ant", "humanoid", "mtu_humanoid", "model_by_name",
           "pendulum", "free_body", "sliding_block", "chain", "muscle_arm", "with_termination",
           "initial_states", "mlp_params", "workload", "WORKLOADS"]
