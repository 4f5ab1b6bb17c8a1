"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package holds only input generation: a counter-based SplitMix64 stream,
binary targets built from geometric primitives (voxel-centre inside tests),
pupil sample tables and the geometry parameters of the benchmark workloads.
It contains none of the projector's arithmetic (no ray tracing, refraction,
sampling, interpolation or attenuation): both the FP64 oracle and the HIP
library receive what is generated here as plain inputs.
"""
from .rng import SplitMix64, splitmix64_outputs
from .pupil import pupil_concentric_jittered, pupil_hex13, concentric_map
from .targets import (
    primitive_target, gaussian_blob_volume, random_config1_target,
    random_config2_target, random_config3_target, fin_stack_target,
)
from .configs import workload, WORKLOADS
from . import cnninit

__all__ = [
    "SplitMix64", "splitmix64_outputs", "pupil_concentric_jittered",
    "pupil_hex13", "concentric_map", "primitive_target",
    "gaussian_blob_volume", "random_config1_target", "random_config2_target",
    "random_config3_target", "fin_stack_target", "workload", "WORKLOADS", "cnninit",
]
