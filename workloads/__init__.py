"""Seeded synthetic inputs shared by the oracle and the GPU path (no method arithmetic)."""
from .scenes import (SHADOW, REFLECT, REFRACT, MAT_REFLECT, MAT_REFRACT, Scene, Workload,
                     make_workload, make_c1, make_c2, make_c3, make_c5, make_frame, make_batch)
