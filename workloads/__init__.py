"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark."""
from .synth import (Box, config0, config1, config2, config3, config4, config5, make, uniform_box,
                    phase_space_hosts,
                    clumpy_box, cubic_lattice, wrap_to_f32, linking_length, SEED_BASE,
                    REINFORCE_SEED, CONFIG3_TAU_FRAC, CONFIG3_K)
