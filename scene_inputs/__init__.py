"""Seeded synthetic scene descriptors shared by the oracle and the HIP path.

This package holds geometry and material *inputs* only (positions, masses,
inertias, meshes, joint frames, drive targets).  It contains none of the
solver's arithmetic: no constraint functions, no NCP functions, no lumped
masses, no contact generation.  Both the FP64 oracle and the GPU library
consume the same `EnvDesc` objects produced here.
"""
from .scenes import (  # noqa: F401
    EnvDesc, SolverParams,
    SHAPE_BOX, SHAPE_CAPSULE, SHAPE_NONE, JOINT_REVOLUTE, JOINT_PRISMATIC,
    NCP_FB, NCP_MIN, RMODE_IDENTITY, RMODE_H2, RMODE_H2_EFFMASS,
    FEM_FULL_PROJECTED, FEM_DIAGONAL, WARM_ZERO, WARM_PREV, WARM_LEARNED, WARM_HYBRID, TET_NEOHOOKEAN, TET_LINEAR,
    box_inertia, capsule_inertia, hex_grid_tets, sphere_tets,
    cube_stack, heavy_stack, stretched_sheet, extension_bar, tet_block_with_boxes, grasp_scene, batched_env, batched_envs,
    particle_on_plane, free_particle, spinning_box, box_on_incline,
    particles_vs_planes_lcp, single_tet, pendulum_drive, round_to_f32,
)
