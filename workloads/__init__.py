"""Seeded synthetic inputs shared by the oracle and the GPU path (no method arithmetic)."""
from .scenes import (SHADOW, REFLECT, REFRACT, KEY_TYPE_ONLY, KEY_SPHERICAL, MAT_REFLECT, MAT_REFRACT, Scene, Workload, unsorted_variant,
                     make_workload, make_shadow_128, make_refl_1024, make_mixed_1080p, make_adjoint_512, make_frame, make_batch)
