"""Seeded synthetic bundle-adjustment inputs shared by the oracle and the HIP path."""
from .problems import (Problem, config0, config1, config2, config4, tiny, ring_problem,
                       walk_problem, cap_problem, project, so3_exp, schur_block_density, mlp_init,
                       cost, relinearize, camera_array, extrinsics_only)

__all__ = ["Problem", "config0", "config1", "config2", "config4", "tiny", "ring_problem",
           "walk_problem", "cap_problem", "project", "so3_exp", "schur_block_density", "mlp_init",
           "cost", "relinearize", "camera_array", "extrinsics_only"]
