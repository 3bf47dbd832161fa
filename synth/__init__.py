"""Seeded synthetic inputs for the tests and the benchmark (no sigma-cut arithmetic)."""
from .beams import (arts_beam_f32, arts_beam_u8, channel_freqs, dispersion_delay_s,  # noqa: F401
                    pulse_track, rng_for, TSAMP_S)
from .workloads import (Step, td, fd, BeamSpec, make_beam, arts1_specs, arts40_specs,  # noqa: F401
                        uneven72_specs, stress16_specs, STEPS_ARTS1, STEPS_ARTS40_MEAN,
                        STEPS_ARTS40_MEDIAN, STEPS_STRESS, UNEVEN_SHAPES)
